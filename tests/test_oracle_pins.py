"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test ties one oracle step to mathematics or to a library routine:
finite-difference moment conditions, exactness on polynomials, lattice-point
counts, scipy's spherical harmonics, a dense direct solve, closed-form
Coulomb energies of Gaussian densities, multipoles of displaced charges,
translation and pair symmetry, and the energy/potential consistency that
follows from the definition of D (Sec. II.C, Eq. Dxx_mlwf).
"""
import math

import numpy as np
import pytest
from scipy.special import erf, sph_harm_y

from oracle import oracle as O
from paper_1911_10630_amd import synth as S

H_C1 = 10.0 * S.ANG / 48


# ---------------------------------------------------------------------------
# Finite-difference stencil (Eq. d2_1)
# ---------------------------------------------------------------------------

def test_fd_weights_moment_conditions():
    w = O.fd_weights()
    s = np.arange(1, 4)
    assert abs(w[0] + 2 * w[1:].sum()) < 1e-15                    # constants
    assert abs(2 * np.sum(w[1:] * s ** 2) - 2.0) < 1e-14          # d2/dx2 of x^2 / 2
    assert abs(np.sum(w[1:] * s ** 4)) < 1e-14                    # no h^2 error term
    assert abs(np.sum(w[1:] * s ** 6)) < 1e-14                    # no h^4 error term
    assert abs(2 * np.sum(w[1:] * s ** 8)) > 1e-3                 # first surviving term: 6th order


def _lattice_count(k):
    r = np.arange(-k, k + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    return int(np.sum(X * X + Y * Y + Z * Z <= k * k))


def test_subdomain_lattice_counts():
    """Points of the PE sphere of radius k*h are the lattice points in a ball of
    radius k: OEIS A000604 (1, 7, 33, 123, 257, 515, 925) and brute force."""
    a000604 = [1, 7, 33, 123, 257, 515, 925]
    h = 0.4
    for k in range(1, 7):
        s = O.Subdomain((40, 40, 40), (40 * h,) * 3, k * h, (k + 3) * h)
        assert s.n_pe == a000604[k] == _lattice_count(k)
        assert s.n_me == _lattice_count(k + 3)


def test_subdomain_small_config_counts_and_order():
    s = O.Subdomain((48, 48, 48), (10 * S.ANG,) * 3, 4 * S.ANG, 5 * S.ANG)
    off = s.offsets()
    d2 = np.sum((off * s.h) ** 2, axis=1)
    pe, sh = off[: s.n_pe], off[s.n_pe:]
    assert np.all(d2[: s.n_pe] <= (4 * S.ANG) ** 2 * (1 + 1e-12))
    assert np.all(d2[s.n_pe:] > (4 * S.ANG) ** 2 * (1 + 1e-12))
    assert np.all(d2[s.n_pe:] <= (5 * S.ANG) ** 2 * (1 + 1e-12))
    # cell clipping: offsets span [-24, 23] on a 48-point axis, R_ME/h = 24
    assert off.min() == -24 and off.max() == 23
    # each block in z, y, x lexicographic order (Alg. 2 loops over the grid)
    for blk in (pe, sh):
        key = (blk[:, 2] * 1000 + blk[:, 1]) * 1000 + blk[:, 0]
        assert np.all(np.diff(key) > 0)
    # the PE sphere is not clipped: symmetric under x -> -x
    assert set(map(tuple, pe)) == set(map(tuple, pe * np.array([-1, 1, 1])))


# ---------------------------------------------------------------------------
# Pair list and pair origin (Step II / Step III, Eq. l2g)
# ---------------------------------------------------------------------------

def test_pair_list_minimum_image_and_strict_cutoff():
    L = 10.0
    C = np.array([[0.5, 5, 5], [9.7, 5, 5], [5, 5, 5], [5, 5, 7.0]])
    pi, pj = O.pair_list(C, (L, L, L), 2.0)
    got = set(zip(pi.tolist(), pj.tolist()))
    # 0-1 are 0.8 apart across the boundary; 2-3 exactly 2.0 apart (strict <)
    assert got == {(0, 0), (0, 1), (1, 1), (2, 2), (3, 3)}
    pi, pj = O.pair_list(C, (L, L, L), 2.0 + 1e-9)
    assert (2, 3) in set(zip(pi.tolist(), pj.tolist()))
    assert list(pi) == sorted(pi)


def test_alg1_hand_worked_examples():
    """Alg. 1 on two cases worked by hand (tests/golden/alg1_unique_pairs.json)."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "alg1_unique_pairs.json")))
    for case in g["cases"]:
        C = np.array(case["centers"], float)
        pi, pj = O.pair_list(C, case["cell"], case["r_pair"])
        assert [[int(a), int(b)] for a, b in zip(pi, pj)] == case["pairs"], case["name"]
        owner, sweeps = O.unique_pair_owners(C, case["cell"], case["r_pair"])
        assert owner.tolist() == case["owner"], case["name"]
        assert sweeps == case["sweeps"], case["name"]


def test_alg1_paper_worked_example():
    """The worked example of the paper's pair-list figure (four orbitals of one
    water molecule, tests/golden/alg1_paper_example.json): Alg. 1 on the
    printed rows gives the printed unique rows and loads, for every order of
    the entries the caption leaves open."""
    import itertools, json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "alg1_paper_example.json")))
    rows = g["L0"]
    n = len(rows)
    for fills in itertools.product(*[itertools.permutations(sorted(set(range(1, n + 1)) - {v for v in r if v}))
                                     for r in rows]):
        L0 = []
        for r, f in zip(rows, fills):
            known = [v for v in r if v is not None]
            L0.append([v - 1 for v in known + list(f)])
        Lu, sweeps = O.refine_pair_rows(L0)
        assert [[v + 1 for v in r] for r in Lu] == g["Lu"], fills
        assert [len(r) for r in Lu] == g["loads"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_alg1_assigns_every_pair_once(seed):
    """Whatever the order of removals, Lu holds each unique pair exactly once
    (in the row of i or of j), every self pair stays with its orbital, and the
    rows that are left hold no pair twice (Sec. III C: all redundancies are
    removed)."""
    rng = np.random.default_rng(seed)
    C = rng.uniform(-5.0, 25.0, size=(60, 3))
    owner, sweeps = O.unique_pair_owners(C, [20.0, 20.0, 20.0], 6.0)
    pi, pj = O.pair_list(C, [20.0, 20.0, 20.0], 6.0)
    assert len(owner) == len(pi) and sweeps >= 2
    assert np.all((owner == pi) | (owner == pj))
    assert np.all(owner[pi == pj] == pi[pi == pj])
    rows = {}
    for p in range(len(pi)):
        other = pj[p] if owner[p] == pi[p] else pi[p]
        rows.setdefault(int(owner[p]), []).append(int(other))
    for i, r in rows.items():
        assert len(r) == len(set(r))
        for j in r:
            if j != i:
                assert i not in rows.get(j, []), (i, j)


def test_alg1_distance_order_balances_the_owners():
    """The paper: sorting each row by distance is what keeps the owners
    balanced; in index order the sweeps pile the pairs onto a few orbitals.
    On the 64-water centres the most-loaded owner has within 10 % of the mean
    with distance order, and well over 1.5x the mean in index order."""
    wl = S.c2_water64()
    for by_distance, bound in ((True, 1.1), (False, 1.5)):
        owner, _ = O.unique_pair_owners(wl.orbitals.centers, wl.cell, wl.r_pair, by_distance=by_distance)
        load = np.bincount(owner, minlength=wl.orbitals.n) - 1       # non-self pairs owned
        ratio = load.max() / load.mean()
        assert (ratio <= bound) if by_distance else (ratio > bound), (by_distance, ratio)


def test_lens_ball_closed_forms():
    """Smallest ball around B(C_i, R_i) cap B(C_j, R_j): equal radii give the
    circle's ball sqrt(R^2 - d^2/4) midway; a ball inside the other is that
    ball; when the intersection holds a great circle of B_i, B_i itself;
    disjoint balls give nothing; the minimum image applies."""
    cell = [40.0, 40.0, 40.0]
    f, rho = O.lens_enclosing_ball([1.0, 2.0, 3.0], [1.0, 2.0, 5.4], 2.0, 2.0, cell)
    assert abs(f - 0.5) < 1e-15 and abs(rho - math.sqrt(4.0 - 1.2 ** 2)) < 1e-14
    assert O.lens_enclosing_ball([0, 0, 0], [1.0, 0, 0], 3.0, 1.0, cell) == (1.0, 1.0)
    assert O.lens_enclosing_ball([0, 0, 0], [2.5, 0, 0], 1.0, 3.0, cell) == (0.0, 1.0)
    assert O.lens_enclosing_ball([0, 0, 0], [3.0, 0, 0], 1.0, 2.0, cell) is None
    f, rho = O.lens_enclosing_ball([0.5, 0, 0], [39.5, 0, 0], 1.0, 1.0, cell)   # 1.0 apart across the boundary
    assert abs(rho - math.sqrt(0.75)) < 1e-14


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_lens_ball_encloses_and_is_tight(seed):
    """Brute force: every sampled point of the lens lies in the ball, and the
    farthest one is within a sampling step of its surface."""
    rng = np.random.default_rng(seed)
    Ri, Rj = rng.uniform(0.8, 3.0, 2)
    d = rng.uniform(abs(Ri - Rj) * 0.5, (Ri + Rj) * 0.95)
    ci, cj = np.zeros(3), np.array([d, 0.0, 0.0])
    f, rho = O.lens_enclosing_ball(ci, cj, Ri, Rj, [100.0] * 3)
    step = 0.02
    r = np.arange(-max(Ri, Rj), max(Ri, Rj) + d + step, step)
    X, Y = np.meshgrid(r, np.arange(0.0, max(Ri, Rj) + step, step), indexing="ij")   # axial symmetry: (x, radial)
    inside = (X ** 2 + Y ** 2 <= Ri ** 2) & ((X - d) ** 2 + Y ** 2 <= Rj ** 2)
    dist = np.sqrt((X[inside] - f * d) ** 2 + Y[inside] ** 2)
    assert dist.max() <= rho * (1 + 1e-12)
    assert dist.max() >= rho - 2 * step


def test_pair_domain_radius_from_the_origin():
    """The radius about the origin g is |g - c| + rho; the self pair's domain
    is the orbital's ball; an empty domain needs nothing."""
    cell, n = [24.0, 24.0, 24.0], [48, 48, 48]                       # h = 0.5
    ci, cj = np.array([5.0, 5.0, 5.0]), np.array([6.0, 5.0, 5.0])
    g = O.pair_origin(ci, cj, cell, n)                               # 5.5 -> grid point 11 (x), 10, 10
    r = O.pair_domain_radius(ci, cj, 2.0, 2.0, g, cell, n, False)
    assert abs(r - math.sqrt(4.0 - 0.25)) < 1e-14                    # g sits on the lens centre
    rs = O.pair_domain_radius(ci, ci, 1.5, 1.5, O.pair_origin(ci, ci, cell, n), cell, n, True)
    assert abs(rs - 1.5) < 1e-14                                     # C_i on a grid point
    assert O.pair_domain_radius(ci, np.array([9.0, 5.0, 5.0]), 1.0, 1.0, g, cell, n, False) == 0.0


def test_pair_classes_cover_the_domain():
    """Each pair's class is the smallest whose radius covers its domain, or
    the largest (counted) when none does."""
    wl = S.c1_small()
    rng = np.random.default_rng(3)
    spreads = rng.uniform(0.6, 1.4, wl.orbitals.n)
    radii = [2.0, 3.0, 4.0]
    cls, capped = O.pair_classes(wl.orbitals.centers, spreads, wl.cell, wl.n_grid, wl.r_pair, 3.0, radii)
    pi, pj = O.pair_list(wl.orbitals.centers, wl.cell, wl.r_pair)
    C = wl.orbitals.centers
    n_cap = 0
    for p, (i, j) in enumerate(zip(pi, pj)):
        g = O.pair_origin(C[i], C[j], wl.cell, wl.n_grid)
        r = O.pair_domain_radius(C[i], C[j], 3.0 * spreads[i], 3.0 * spreads[j], g, wl.cell, wl.n_grid, i == j)
        k = cls[p]
        if r > radii[-1]:
            assert k == 2
            n_cap += 1
        else:
            assert radii[k] >= r and (k == 0 or radii[k - 1] < r)
    assert n_cap == capped
    assert len(set(cls.tolist())) == 3                               # all classes in use here


def test_pair_origin_wraps_and_rounds():
    L, N = 10.0, 20                                    # h = 0.5
    # midpoint 0.1 -> grid 0
    assert list(O.pair_origin([0.5, 5, 5], [9.7, 5, 5], (L,) * 3, (N,) * 3)) == [0, 10, 10]
    # midpoint -0.2 wraps to 9.8 -> 19.6 -> 20 -> 0 (non-negative MOD)
    assert list(O.pair_origin([0.1, 5, 5], [9.5, 5, 5], (L,) * 3, (N,) * 3)) == [0, 10, 10]
    # half-way value 2.25/0.5 = 4.5 rounds away from zero -> 5
    assert list(O.pair_origin([2.0, 5, 5], [2.5, 5, 5], (L,) * 3, (N,) * 3)) == [5, 10, 10]


# ---------------------------------------------------------------------------
# Operator and CG (Eqs. d2_1, pe_mat_red)
# ---------------------------------------------------------------------------

def test_operator_exact_on_degree7_polynomials():
    """-A f + (shell part) f = full stencil Laplacian, exact for degree <= 7."""
    h = 0.37
    s = O.Subdomain((40, 40, 40), (40 * h,) * 3, 6 * h, 9 * h)
    off = s.offsets().astype(np.float64) * h / 3.0      # keep values O(1)
    x, y, z = off[:, 0], off[:, 1], off[:, 2]
    f = 1 + x - 2 * y * z + x ** 2 * y + 0.5 * z ** 4 - 0.3 * x ** 3 * y ** 2 * z + 0.1 * x ** 7 - 0.2 * y ** 5 * z ** 2
    # analytic Laplacian; the coordinates were scaled by 1/3, so divide by 9
    f_xx = 2 * y - 1.8 * x * y ** 2 * z + 4.2 * x ** 5
    f_yy = -0.6 * x ** 3 * z - 4.0 * y ** 3 * z ** 2
    f_zz = 6.0 * z ** 2 - 0.4 * y ** 5
    lap = (f_xx + f_yy + f_zz) / 9.0
    lhs = -s.apply_A(f[: s.n_pe]) + s.rhs(np.zeros(s.n_pe), f[s.n_pe:])
    assert np.max(np.abs(lhs - lap[: s.n_pe])) < 1e-9 * np.max(np.abs(lap))


def test_cg_matches_dense_solve_on_tiny_sphere():
    h = 0.5
    s = O.Subdomain((32, 32, 32), (32 * h,) * 3, 6 * h, 9 * h)
    n = s.n_pe
    assert n == 925
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        A[:, k] = s.apply_A(e)
    assert np.array_equal(A, A.T)
    np.linalg.cholesky(A)                                    # SPD
    rng = np.random.default_rng(7)
    b = rng.normal(size=n)
    x_ref = np.linalg.solve(A, b)
    x, it, conv, rel = s.cg(b, tol=1e-14)
    assert conv and rel < 1e-13
    assert np.max(np.abs(x - x_ref)) < 1e-11 * np.max(np.abs(x_ref))


# ---------------------------------------------------------------------------
# Spherical harmonics and multipoles (Eqs. mepole, me)
# ---------------------------------------------------------------------------

def test_ylm_matches_scipy():
    rng = np.random.default_rng(3)
    for _ in range(20):
        th, ph = rng.uniform(0, np.pi), rng.uniform(-np.pi, np.pi)
        for l in range(7):
            for m in range(-l, l + 1):
                ref = complex(sph_harm_y(l, m, th, ph))
                assert abs(O.ylm(l, m, th, ph) - ref) < 1e-13


def _gauss_on(off, h, d, p, q=1.0):
    r = off * h - np.asarray(d)
    return q * (p / np.pi) ** 1.5 * np.exp(-p * np.sum(r * r, axis=1))


def test_moments_of_displaced_gaussian():
    """A spherical charge q at d has Q_lm = q |d|^l conj(Y_lm(dhat))."""
    s = O.Subdomain((48, 48, 48), (10 * S.ANG,) * 3, 4 * S.ANG, 5 * S.ANG)
    off = s.offsets()[: s.n_pe].astype(np.float64)
    d = np.array([0.31, -0.22, 0.17])
    p, q = 1.1, 0.8
    Q = s.moments(_gauss_on(off, s.h, d, p, q))
    dn = np.linalg.norm(d)
    th, ph = math.acos(d[2] / dn), math.atan2(d[1], d[0])
    for l in range(7):
        for m in range(-l, l + 1):
            ref = q * dn ** l * np.conj(complex(sph_harm_y(l, m, th, ph)))
            assert abs(Q[l * l + l + m] - ref) < 1e-12, (l, m)


def test_shell_potential_matches_coulomb():
    s = O.Subdomain((48, 48, 48), (10 * S.ANG,) * 3, 4 * S.ANG, 5 * S.ANG)
    off = s.offsets().astype(np.float64)
    d = np.array([0.3, -0.1, 0.2])
    p, q = 1.3, 1.0
    Q = s.moments(_gauss_on(off[: s.n_pe], s.h, d, p, q))
    v = s.shell_potential(Q)
    r = np.linalg.norm(off[s.n_pe:] * s.h - d, axis=1)
    v_ref = q * erf(math.sqrt(p) * r) / r
    # l <= 6 truncation error ~ (|d|/r)^7 ~ 1e-10
    assert np.max(np.abs(v - v_ref) / v_ref) < 1e-8


# ---------------------------------------------------------------------------
# Whole pair solve against closed forms
# ---------------------------------------------------------------------------

def _s_orbital_grid(n, L, c, alpha):
    h = L / n
    ax = np.arange(n) * h
    d = [ax - c[k] for k in range(3)]
    d = [dd - L * np.round(dd / L) for dd in d]
    g = np.exp(-alpha * d[2][:, None, None] ** 2) * np.exp(-alpha * d[1][None, :, None] ** 2) \
        * np.exp(-alpha * d[0][None, None, :] ** 2)
    return (2 * alpha / np.pi) ** 0.75 * g


@pytest.mark.parametrize("n", [48, 96])
def test_self_energy_of_s_gaussian(n):
    """Self pair of a normalized s Gaussian: e = (rho|rho) = 2 sqrt(alpha/pi)."""
    L, alpha = 10 * S.ANG, 0.8
    c = np.array([L / 2, L / 2, L / 2])
    phi = _s_orbital_grid(n, L, c, alpha)
    s = O.Subdomain((n,) * 3, (L,) * 3, 4 * S.ANG, 5 * S.ANG)
    gc = O.pair_origin(c, c, (L,) * 3, (n,) * 3)
    r = s.solve_pair(phi, phi, gc, tol=1e-12)
    exact = 2 * math.sqrt(alpha / math.pi)
    err = abs(r["e"] - exact) / exact
    # 6th-order FD error: 2x the level measured for p = 1.6 at these spacings
    assert err < {48: 2.2e-4, 96: 4e-6}[n], err
    test_self_energy_of_s_gaussian.errs = getattr(test_self_energy_of_s_gaussian, "errs", {})
    test_self_energy_of_s_gaussian.errs[n] = err


def test_self_energy_converges_at_sixth_order():
    errs = getattr(test_self_energy_of_s_gaussian, "errs", {})
    if len(errs) < 2:
        pytest.skip("needs both spacings from the previous test")
    assert errs[48] / errs[96] > 30.0                         # ~2^6 asymptotically


def test_two_center_product_across_boundary():
    """rho_ab = S_ab * normalized Gaussian of exponent a+b centred at
    P = (aA + bB)/(a+b); (rho|rho) = S_ab^2 sqrt(2p/pi).  Centres straddle
    the periodic boundary, so the gather wraps."""
    n, L = 48, 10 * S.ANG
    a, b = 0.7, 0.9
    A = np.array([0.4, 9.0, 18.5])
    B = np.array([18.2, 9.6, 0.3])
    pa = _s_orbital_grid(n, L, A, a)
    pb = _s_orbital_grid(n, L, B, b)
    s = O.Subdomain((n,) * 3, (L,) * 3, 4 * S.ANG, 5 * S.ANG)
    gc = O.pair_origin(A, B, (L,) * 3, (n,) * 3)
    r = s.solve_pair(pa, pb, gc, tol=1e-12)
    dAB = B - A
    dAB -= L * np.round(dAB / L)
    mu = a * b / (a + b)
    Sab = (4 * a * b / (a + b) ** 2) ** 0.75 * math.exp(-mu * float(dAB @ dAB))
    exact = Sab ** 2 * math.sqrt(2 * (a + b) / math.pi)
    assert abs(r["e"] - exact) / exact < 3e-4
    # the monopole of the pair density is the overlap
    assert abs(r["Q"][0] * math.sqrt(4 * math.pi) - Sab) < 1e-10


# ---------------------------------------------------------------------------
# Invariants of the whole step
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c1_result():
    wl = S.c1_small()
    phi = S.orbitals_np(wl)
    E, D, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi)
    return wl, phi, E, D, out


def test_c1_pairs_and_convergence(c1_result):
    wl, phi, E, D, out = c1_result
    assert len(out["e"]) == 60
    assert np.all(out["converged"] == 1)
    assert np.all(out["relres"] < 1e-9)
    assert E < 0
    # E is the weighted sum of the pair energies
    w = np.where(out["i"] == out["j"], 1.0, 2.0)
    assert abs(E + np.sum(w * out["e"])) < 1e-12 * abs(E)


def test_translation_by_grid_vector(c1_result):
    wl, phi, E, D, out = c1_result
    k = np.array([3, -5, 7])
    C = np.mod(wl.orbitals.centers + k * np.array(wl.h), wl.cell[0])
    phis = np.roll(phi, shift=(k[2], k[1], k[0]), axis=(1, 2, 3))
    E2, D2, _ = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, C, phis)
    assert abs(E2 - E) <= 1e-13 * abs(E)
    Dr = np.roll(D, shift=(k[2], k[1], k[0]), axis=(1, 2, 3))
    assert np.max(np.abs(D2 - Dr)) <= 1e-13 * np.max(np.abs(D))


def test_pair_potential_symmetric(c1_result):
    wl, phi, *_ = c1_result
    s = O.Subdomain(wl.n_grid, wl.cell, wl.r_pe[1], wl.r_me[1])
    C = wl.orbitals.centers
    gc = O.pair_origin(C[2], C[5], wl.cell, wl.n_grid)
    a = s.solve_pair(phi[2], phi[5], gc)
    b = s.solve_pair(phi[5], phi[2], gc)
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["vsh"], b["vsh"])


@pytest.mark.slow
def test_energy_potential_consistency(c1_result):
    """dE/d eps along phi_k + eps*eta equals -4 h^3 <eta, D^k> (real orbitals)."""
    wl, phi, E, D, out = c1_result
    h3 = float(np.prod(wl.h))
    k = 3
    c = wl.orbitals.centers[k]
    eta = _s_orbital_grid(wl.n_grid[0], wl.cell[0], c, 1.5)
    eps = 1e-3
    Es = []
    for sgn in (+1, -1):
        p2 = phi.copy()
        p2[k] += sgn * eps * eta
        Es.append(O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, p2,
                        tol=1e-13, want_D=False)[0])
    fd = (Es[0] - Es[1]) / (2 * eps)
    _, D13, _ = O.exx(wl.n_grid, wl.cell, wl.r_pair, wl.r_pe, wl.r_me, wl.orbitals.centers, phi, tol=1e-13)
    an = -4 * h3 * float(np.sum(eta * D13[k]))
    assert abs(fd - an) < 1e-5 * abs(an), (fd, an)


def test_per_class_pipeline_reduces_to_the_two_fixed_classes(c1_result):
    """The per-pair-class accumulation (Python, one Subdomain per class)
    given the fixed classes (self pairs on class 0, the others on class 1)
    reproduces the C pipeline's E and D exactly: same pair solves, same
    pair order of the D sums."""
    wl, phi, E, D, out = c1_result
    pi, pj = O.pair_list(wl.orbitals.centers, wl.cell, wl.r_pair)
    cls = (pi != pj).astype(np.int32)
    classes = [(wl.r_pe[0], wl.r_me[0]), (wl.r_pe[1], wl.r_me[1])]
    E2, D2, o2 = O.exx_classed(wl.n_grid, wl.cell, wl.r_pair, classes, cls, wl.orbitals.centers, phi)
    assert E2 == E
    assert np.array_equal(D2, D)
    assert np.array_equal(o2["e"], out["e"])


def test_orthogonal_mixing_of_the_orbitals():
    """E_xx = -sum over ordered pairs of (rho_ij | rho_ij) is invariant under
    an orthogonal mixing phi -> U phi, and D transforms as D -> U D, when
    every pair is solved by the same linear operator: all centres at one
    point (one pair origin) and equal self / non-self radii.  Exact up to the
    CG tolerance."""
    n, cell = (32, 32, 32), (12.0, 12.0, 12.0)
    rng = np.random.default_rng(5)
    C = np.tile([6.0, 6.0, 6.0], (4, 1))
    u = rng.normal(size=(4, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    wl = S.custom(n, cell, C, kind=[0, 1, 0, 1], alpha=rng.uniform(1.2, 2.0, 4), u=u,
                  a=rng.uniform(-0.2, 0.2, (4, 3)), r_pair=1.0, r_pe=4.0, r_me=5.5)
    phi = S.orbitals_np(wl)
    E, D, _ = O.exx(n, cell, wl.r_pair, wl.r_pe, wl.r_me, C, phi)
    U, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    E2, D2, _ = O.exx(n, cell, wl.r_pair, wl.r_pe, wl.r_me, C, np.einsum("ik,k...->i...", U, phi))
    assert abs(E2 - E) <= 1e-10 * abs(E)
    assert np.abs(D2 - np.einsum("ik,k...->i...", U, D)).max() <= 1e-9 * np.abs(D).max()


def test_energy_converges_with_the_subdomain_radius():
    """The paper's convergence test (Sec. IV A): the self-pair energy of one
    diffuse s orbital approaches its large-domain value monotonically as
    R_PE grows (R_ME = R_PE + 1.5 bohr) until the solver's tolerance."""
    n, cell = (32, 32, 32), (12.0, 12.0, 12.0)
    C = np.array([[6.0, 6.0, 6.0]])
    wl = S.custom(n, cell, C, alpha=[0.9], r_pair=1.0)
    phi = S.orbitals_np(wl)
    radii = [2.0, 2.5, 3.0, 3.5, 4.5]
    E = [O.exx(n, cell, 1.0, r, r + 1.5, C, phi, want_D=False)[0] for r in radii]
    err = [abs(e - E[-1]) for e in E[:-1]]
    assert all(a > b for a, b in zip(err, err[1:])), err
    assert err[0] > 1e-3 * abs(E[-1]) and err[-1] < 1e-7 * abs(E[-1])


# ---------------------------------------------------------------------------
# The explicit-pair-list leg (the benchmark's CPU baseline and the sampled
# full-size checks run it) and the wrap of the per-pair domain radius
# ---------------------------------------------------------------------------

def test_solve_pairs_reproduces_the_whole_step_per_pair():
    """solve_pairs on every pair of the small workload, in shuffled order and
    with self and non-self pairs on different radii (4 A and 3.4 A), returns
    exactly the per-pair energy, iterations, flag and residual of the whole
    step (Steps III-V): the orbital pointer table, the class of each pair
    and the result order all line up."""
    wl = S.c1_small()
    r_pe, r_me = (4.0 * S.ANG, 3.4 * S.ANG), (5.0 * S.ANG, 4.4 * S.ANG)
    phi = S.orbitals_np(wl)
    E, _, out = O.exx(wl.n_grid, wl.cell, wl.r_pair, r_pe, r_me, wl.orbitals.centers, phi, want_D=False)
    perm = np.random.default_rng(7).permutation(len(out["i"]))
    res = O.solve_pairs(wl.n_grid, wl.cell, r_pe, r_me, wl.orbitals.centers, {k: phi[k] for k in range(len(phi))},
                        out["i"][perm], out["j"][perm], nthreads=4)
    for key in ("e", "iters", "converged", "relres"):
        assert np.array_equal(res[key], out[key][perm]), key
    assert np.sum(out["i"] == out["j"]) == 16


def test_solve_pairs_on_rounded_box_orbitals_matches_each_class():
    """solve_pairs on FP32-rounded orbitals that live on local boxes (zero
    outside, as the 512-water workload stores them), given only the orbitals
    the sampled pairs touch, equals the single-pair pipeline of the class the
    header names for each pair: [0] for self pairs, [1] for the others."""
    wl = S.c1_boxed()
    r_pe, r_me = (4.0 * S.ANG, 3.5 * S.ANG), (5.0 * S.ANG, 4.5 * S.ANG)
    C = wl.orbitals.centers
    n, box, h = np.asarray(wl.n_grid), np.asarray(wl.box), np.asarray(wl.h)
    # box origin: the grid point nearest the centre minus half the box
    origins = [np.mod(np.floor(np.mod(c, wl.cell[0]) / h + 0.5).astype(int) - box // 2, n) for c in C]
    pi, pj = O.pair_list(C, wl.cell, wl.r_pair)
    rng = np.random.default_rng(5)
    pick = np.concatenate([rng.choice(np.nonzero(pi == pj)[0], 2, replace=False),
                           rng.choice(np.nonzero(pi != pj)[0], 4, replace=False)])
    orbs = sorted(set(pi[pick].tolist()) | set(pj[pick].tolist()))
    vals = S.embed_boxes(S.orbitals_np(wl, orbs, origins=origins), [origins[k] for k in orbs], wl.n_grid)
    vals = vals.astype(np.float32).astype(np.float64)
    phis = dict(zip(orbs, vals))
    assert np.count_nonzero(vals[0]) < vals[0].size            # the boxes leave zeros
    res = O.solve_pairs(wl.n_grid, wl.cell, r_pe, r_me, C, phis, pi[pick], pj[pick], nthreads=2)
    subs = [O.Subdomain(wl.n_grid, wl.cell, r_pe[k], r_me[k]) for k in (0, 1)]
    for t, p in enumerate(pick):
        i, j = int(pi[p]), int(pj[p])
        ref = subs[0 if i == j else 1].solve_pair(phis[i], phis[j], O.pair_origin(C[i], C[j], wl.cell, wl.n_grid))
        assert res["e"][t] == ref["e"] and res["iters"][t] == ref["iters"], (i, j)
        assert res["relres"][t] == ref["relres"] and res["converged"][t] == ref["converged"]


def test_pair_domain_radius_wraps_across_the_boundary():
    """Worked by hand, L = 10, N = 20 (h = 0.5): C_i = (9.8, 2.5, 2.5) and
    C_j = (0.3, 2.5, 2.5) are 0.5 apart through the face x = 0.  The
    midpoint 10.05 wraps to 0.05, so the origin is grid point (0, 5, 5);
    g - C_i is 0.2 along x only after the minimum-image wrap (-9.8 without
    it).  With R_i = R_j = 1 the lens ball sits at C_i + 0.25 with radius
    sqrt(1 - 0.25^2), so the radius is 0.05 + sqrt(0.9375); the self pair of
    i needs 0.2 + R_i."""
    cell, n = (10.0, 10.0, 10.0), (20, 20, 20)
    ci, cj = np.array([9.8, 2.5, 2.5]), np.array([0.3, 2.5, 2.5])
    g = O.pair_origin(ci, cj, cell, n)
    assert list(g) == [0, 5, 5]
    r = O.pair_domain_radius(ci, cj, 1.0, 1.0, g, cell, n, False)
    assert abs(r - (0.05 + math.sqrt(0.9375))) < 1e-12, r
    gs = O.pair_origin(ci, ci, cell, n)                              # 19.6 -> 20 -> 0
    assert list(gs) == [0, 5, 5]
    rs = O.pair_domain_radius(ci, ci, 1.0, 1.0, gs, cell, n, True)
    assert abs(rs - 1.2) < 1e-12, rs
    # the same pair seen from j: the lens centre is C_j - 0.25, the origin
    # the same grid point, 0.3 - 0.25 = 0.05 from it
    r2 = O.pair_domain_radius(cj, ci, 1.0, 1.0, g, cell, n, False)
    assert abs(r2 - r) < 1e-12


def test_solve_pairs_classed_matches_each_class_and_the_two_fixed_classes(c1_result):
    """Each pair on its own class equals that class's single-pair pipeline bit
    for bit; with two classes chosen self -> 0, other -> 1 it equals the
    fixed-class explicit-list solve."""
    wl, phi, E, D, out = c1_result
    C = wl.orbitals.centers
    classes = [(3.0, 5.0), (4.0, 6.0), (5.5, 7.5)]
    rng = np.random.default_rng(21)
    pick = rng.choice(len(out["i"]), 7, replace=False)
    pi, pj = out["i"][pick], out["j"][pick]
    cls = rng.integers(0, 3, len(pick)).astype(np.int32)
    phis = {k: phi[k] for k in range(len(phi))}
    res = O.solve_pairs_classed(wl.n_grid, wl.cell, classes, C, phis, pi, pj, cls, nthreads=4)
    subs = [O.Subdomain(wl.n_grid, wl.cell, a, b) for a, b in classes]
    for t in range(len(pick)):
        i, j = int(pi[t]), int(pj[t])
        ref = subs[cls[t]].solve_pair(phi[i], phi[j], O.pair_origin(C[i], C[j], wl.cell, wl.n_grid))
        assert res["e"][t] == ref["e"] and res["iters"][t] == ref["iters"] and res["relres"][t] == ref["relres"]
    two = [(wl.r_pe[0], wl.r_me[0]), (wl.r_pe[1], wl.r_me[1])]
    c2 = np.where(pi == pj, 0, 1).astype(np.int32)
    a = O.solve_pairs_classed(wl.n_grid, wl.cell, two, C, phis, pi, pj, c2, nthreads=4)
    b = O.solve_pairs(wl.n_grid, wl.cell, wl.r_pe, wl.r_me, C, phis, pi, pj, nthreads=4)
    for key in ("e", "iters", "converged", "relres"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("k", [0, 7])
def test_dxx_orbital_equals_the_whole_step(c1_result, k):
    """D^k from the list of k's pairs in pair order equals the whole step's
    D^k bit for bit (same solves, same summation order), and the orbital's
    partners' phi are the only ones it reads."""
    wl, phi, E, D, out = c1_result
    C = wl.orbitals.centers
    sel = np.nonzero((out["i"] == k) | (out["j"] == k))[0]
    pi, pj = out["i"][sel], out["j"][sel]
    touch = sorted(set(pi.tolist()) | set(pj.tolist()))
    two = [(wl.r_pe[0], wl.r_me[0]), (wl.r_pe[1], wl.r_me[1])]
    cls = np.where(pi == pj, 0, 1).astype(np.int32)
    Dk = O.dxx_orbital(wl.n_grid, wl.cell, two, C, {q: phi[q] for q in touch}, pi, pj, cls, k, nthreads=4)
    assert np.array_equal(Dk, D[k])
    assert len(sel) >= 3


def test_water64_golden_file_is_the_oracle_step():
    """tests/golden/water64_oracle.npz (the oracle's whole 64-water step, written
    by tests/golden/make_water64_oracle.py) holds the workload's pair list in
    the oracle's order, E_xx as the weighted sum of its pair energies
    (Eq. exx_omega), and, re-solved here, bit for bit the oracle's per-pair
    results on a self pair and two other pairs."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "water64_oracle.npz")
    if not os.path.exists(path):
        pytest.skip("golden file not written")
    g = np.load(path, allow_pickle=False)
    wl = S.c2_water64()
    pi, pj = O.pair_list(wl.orbitals.centers, wl.cell, wl.r_pair)
    assert np.array_equal(g["i"], pi) and np.array_equal(g["j"], pj)
    w = np.where(g["i"] == g["j"], 1.0, 2.0)
    assert abs(float(g["E"]) + np.sum(w * g["e"])) <= 1e-13 * abs(float(g["E"]))
    assert np.all(g["converged"] == 1) and g["relres"].max() <= 1e-10 * (1 + 1e-4)
    pick = np.array([int(np.nonzero(g["i"] == g["j"])[0][3]), 1234, 8765])
    need = sorted(set(g["i"][pick].tolist()) | set(g["j"][pick].tolist()))
    phis = dict(zip(need, S.orbitals_np(wl, need)))
    res = O.solve_pairs(wl.n_grid, wl.cell, wl.r_pe, wl.r_me, wl.orbitals.centers, phis, g["i"][pick], g["j"][pick],
                        tol=wl.cg_rtol, nthreads=3)
    for key in ("e", "iters", "converged", "relres"):
        assert np.array_equal(res[key], g[key][pick]), key
