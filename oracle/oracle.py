"""ctypes wrapper of the plain FP64 CPU oracle (exx_oracle.c).

Test infrastructure only: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "exx_oracle.c")
_LIB = os.path.join(_HERE, "libexx_oracle.so")
NLM = 49

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.o_pair_list.restype = C.c_int
        L.o_pair_list.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, C.c_void_p, C.c_void_p]
        L.o_pair_origin.restype = None
        L.o_pair_origin.argtypes = [_dp, _dp, _dp, _ip, _ip]
        L.o_sub_build.restype = C.c_int
        L.o_sub_build.argtypes = [_ip, _dp, C.c_double, C.c_double, C.POINTER(C.c_void_p)]
        L.o_sub_free.argtypes = [C.c_void_p]
        L.o_sub_info.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), _ip, _ip]
        L.o_sub_offsets.argtypes = [C.c_void_p, _ip]
        L.o_apply_A.argtypes = [C.c_void_p, _dp, _dp]
        L.o_rhs.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.o_moments.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.o_shell_potential.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.o_cg.restype = C.c_int
        L.o_cg.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.POINTER(C.c_int),
                           C.POINTER(C.c_double)]
        L.o_ylm_reim.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.o_fd_weight.restype = C.c_double
        L.o_fd_weight.argtypes = [C.c_int]
        L.o_solve_pair.restype = C.c_int
        L.o_solve_pair.argtypes = [C.c_void_p, _dp, _dp, _ip, C.c_double, C.c_int] + [C.c_void_p] * 6 + [
            C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.o_exx.restype = C.c_long
        L.o_exx.argtypes = [_ip, _dp, C.c_double, _dp, _dp, C.c_int, _dp, _dp, C.c_double, C.c_int,
                            C.c_int, C.POINTER(C.c_double), C.c_void_p, C.c_long] + [C.c_void_p] * 6
        L.o_solve_pairs.restype = C.c_int
        L.o_solve_pairs.argtypes = [_ip, _dp, _dp, _dp, _dp, C.c_void_p, C.c_int, _ip, _ip, C.c_double,
                                    C.c_int, C.c_int, _dp, _ip, _ip, _dp]
        L.o_solve_pairs_classed.restype = C.c_int
        L.o_solve_pairs_classed.argtypes = [_ip, _dp, C.c_int, _dp, _dp, _dp, C.c_void_p, C.c_int, _ip, _ip, _ip,
                                            C.c_double, C.c_int, C.c_int, _dp, _ip, _ip, _dp]
        L.o_dxx_orbital.restype = C.c_int
        L.o_dxx_orbital.argtypes = [_ip, _dp, C.c_int, _dp, _dp, _dp, C.c_void_p, C.c_int, _ip, _ip, _ip, C.c_int,
                                    C.c_double, C.c_int, C.c_int, _dp]
        _lib = L
    return _lib


def _i3(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.int32).reshape(3))


def _d3(v):
    return np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(3))


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def fd_weights():
    return np.array([lib().o_fd_weight(s) for s in range(4)])


def ylm(l: int, m: int, theta: float, phi: float) -> complex:
    re, im = C.c_double(), C.c_double()
    lib().o_ylm_reim(l, m, theta, phi, C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def pair_list(centers, cell, r_pair):
    L = lib()
    Cc = np.ascontiguousarray(centers, dtype=np.float64)
    n = Cc.shape[0]
    np_ = L.o_pair_list(n, Cc.ravel(), _d3(cell), float(r_pair), 0, None, None)
    pi = np.zeros(np_, np.int32)
    pj = np.zeros(np_, np.int32)
    L.o_pair_list(n, Cc.ravel(), _d3(cell), float(r_pair), np_, _ptr(pi), _ptr(pj))
    return pi, pj


def _nint(v: float) -> int:
    """Nearest integer, halves away from zero (as the C oracle's o_nint)."""
    return int(math.floor(v + 0.5)) if v >= 0.0 else -int(math.floor(-v + 0.5))


def min_image_d2(ci, cj, cell) -> float:
    """Squared minimum-image distance |C_j - C_i|^2: per axis d = C_j - C_i,
    d -= L nint(d / L), summed over x, y, z in that order (plain FP64)."""
    s = 0.0
    for a in range(3):
        d = float(cj[a]) - float(ci[a])
        d -= float(cell[a]) * float(_nint(d / float(cell[a])))
        s += d * d
    return s


def unique_pair_owners(centers, cell, r_pair, by_distance=True):
    """Alg. 1 (Sec. III C): the unique pair list Lu refined from the
    non-unique list L0, given as the owner of every pair.

    L0 row i lists every orbital that overlaps i (the pair criterion of
    Step II), i itself included, ordered by distance from i; distances are
    compared as the squared minimum-image length, ties by index (the paper
    orders by |C_i - C_j| and leaves ties open).  See refine_pair_rows for
    the refinement itself.

    by_distance=False orders each row by index instead, the ordering the
    paper warns against (it unbalances the owners).

    Returns (owner, sweeps): owner[p] for the pairs of pair_list() in its
    order, and the number of sweeps including the last, empty one.
    """
    Cc = np.asarray(centers, dtype=np.float64)
    pi, pj = pair_list(Cc, cell, r_pair)
    n = Cc.shape[0]
    rows = [[] for _ in range(n)]
    for i, j in zip(pi.tolist(), pj.tolist()):
        d2 = min_image_d2(Cc[i], Cc[j], cell)
        rows[i].append((d2, j))
        if j != i:
            rows[j].append((d2, i))
    L0 = [[j for _, j in (sorted(r) if by_distance else sorted(r, key=lambda t: t[1]))] for r in rows]
    Lu, sweeps = refine_pair_rows(L0)
    member = [set(r) for r in Lu]
    owner = np.array([i if j in member[i] else j for i, j in zip(pi.tolist(), pj.tolist())], np.int32)
    return owner, sweeps


def refine_pair_rows(L0):
    """Alg. 1 on explicit rows: L0[i] lists orbital i's overlapping orbitals
    (i among them) in the order the sweeps scan them.  Returns (Lu, sweeps):
    the refined rows, in their original order with the removed entries
    dropped, and the number of sweeps including the last, empty one.

    The rule, as the paper's prose states it: an unordered pair {i, j} is
    redundant while it is listed both in row i and in row j.  A sweep takes
    the orbitals in index order, and each orbital i settles the first
    redundant pair of its row, in the row's order: i keeps it and j's row
    drops i.  Sweeps repeat until one settles nothing.  Here every pair
    carries a holder: "both" while redundant, else the one row that still
    lists it; a self pair is held by its orbital from the start.
    """
    n = len(L0)
    listed = [set(r) for r in L0]
    holder = {}
    for i in range(n):
        for j in L0[i]:
            key = (min(i, j), max(i, j))
            if i == j:
                holder[key] = i
            elif key not in holder:
                holder[key] = "both" if i in listed[j] else i
    sweeps = 0
    while True:
        sweeps += 1
        settled = 0
        for i in range(n):
            for j in L0[i]:
                key = (min(i, j), max(i, j))
                if holder[key] == "both":
                    holder[key] = i
                    settled += 1
                    break
        if settled == 0:
            break
    Lu = [[j for j in L0[i] if holder[(min(i, j), max(i, j))] == i] for i in range(n)]
    return Lu, sweeps


def pair_origin(ci, cj, cell, n):
    gc = np.zeros(3, np.int32)
    lib().o_pair_origin(_d3(ci), _d3(cj), _d3(cell), _i3(n), gc)
    return gc


class Subdomain:
    """One proto-subdomain class (PE sphere + ME shell), Alg. 2."""

    def __init__(self, n, cell, r_pe, r_me):
        self._h = C.c_void_p()
        rc = lib().o_sub_build(_i3(n), _d3(cell), float(r_pe), float(r_me), C.byref(self._h))
        if rc != 0:
            raise ValueError(f"o_sub_build failed ({rc})")
        npe, nme = C.c_int(), C.c_int()
        blo, bhi = np.zeros(3, np.int32), np.zeros(3, np.int32)
        lib().o_sub_info(self._h, C.byref(npe), C.byref(nme), blo, bhi)
        self.n_pe, self.n_me = npe.value, nme.value
        self.n_shell = self.n_me - self.n_pe
        self.blo, self.bhi = blo, bhi
        self.h = np.asarray(cell, np.float64) / np.asarray(n, np.float64)
        self.n = np.asarray(n)

    def __del__(self):
        if getattr(self, "_h", None) and lib is not None:
            try:
                lib().o_sub_free(self._h)
            except Exception:
                pass

    def offsets(self) -> np.ndarray:
        off = np.zeros((self.n_me, 3), np.int32)
        lib().o_sub_offsets(self._h, off.reshape(-1))
        return off

    def apply_A(self, x):
        y = np.zeros(self.n_pe)
        lib().o_apply_A(self._h, np.ascontiguousarray(x, np.float64), y)
        return y

    def rhs(self, rho, vsh):
        b = np.zeros(self.n_pe)
        lib().o_rhs(self._h, np.ascontiguousarray(rho, np.float64),
                    np.ascontiguousarray(vsh, np.float64) if self.n_shell else np.zeros(1), b)
        return b

    def moments(self, rho):
        re, im = np.zeros(NLM), np.zeros(NLM)
        lib().o_moments(self._h, np.ascontiguousarray(rho, np.float64), re, im)
        return re + 1j * im

    def shell_potential(self, Q):
        v = np.zeros(max(self.n_shell, 1))
        lib().o_shell_potential(self._h, np.ascontiguousarray(Q.real), np.ascontiguousarray(Q.imag), v)
        return v[: self.n_shell]

    def cg(self, b, tol=1e-10, maxit=100000):
        x = np.zeros(self.n_pe)
        conv, rel = C.c_int(), C.c_double()
        it = lib().o_cg(self._h, np.ascontiguousarray(b, np.float64), x, tol, maxit, C.byref(conv), C.byref(rel))
        return x, it, bool(conv.value), rel.value

    def solve_pair(self, phi_i, phi_j, gc, tol=1e-10, maxit=100000):
        """Full pair pipeline; returns a dict of every intermediate."""
        x = np.zeros(self.n_pe)
        vsh = np.zeros(max(self.n_shell, 1))
        Qre, Qim = np.zeros(NLM), np.zeros(NLM)
        rho = np.zeros(self.n_pe)
        b = np.zeros(self.n_pe)
        e, it, conv, rel = C.c_double(), C.c_int(), C.c_int(), C.c_double()
        lib().o_solve_pair(self._h, np.ascontiguousarray(phi_i, np.float64).reshape(-1),
                           np.ascontiguousarray(phi_j, np.float64).reshape(-1), _i3(gc), tol, maxit,
                           _ptr(x), _ptr(vsh), _ptr(Qre), _ptr(Qim), _ptr(rho), _ptr(b),
                           C.byref(e), C.byref(it), C.byref(conv), C.byref(rel))
        return dict(x=x, vsh=vsh[: self.n_shell], Q=Qre + 1j * Qim, rho=rho, b=b, e=e.value,
                    iters=it.value, converged=bool(conv.value), relres=rel.value)


def exx(n, cell, r_pair, r_pe, r_me, centers, phi, tol=1e-10, maxit=100000, nthreads=0, want_D=True):
    """Whole step: returns (E, D or None, per-pair dict)."""
    L = lib()
    Cc = np.ascontiguousarray(centers, np.float64)
    n_orb = Cc.shape[0]
    phi = np.ascontiguousarray(phi, np.float64)
    pi, pj = pair_list(Cc, cell, r_pair)
    npairs = len(pi)
    out = dict(i=np.zeros(npairs, np.int32), j=np.zeros(npairs, np.int32), e=np.zeros(npairs),
               iters=np.zeros(npairs, np.int32), converged=np.zeros(npairs, np.int32),
               relres=np.zeros(npairs))
    D = np.zeros_like(phi) if want_D else None
    E = C.c_double()
    rpe = np.ascontiguousarray(np.broadcast_to(np.asarray(r_pe, np.float64), (2,)))
    rme = np.ascontiguousarray(np.broadcast_to(np.asarray(r_me, np.float64), (2,)))
    rc = L.o_exx(_i3(n), _d3(cell), float(r_pair), rpe, rme, n_orb, Cc.ravel(), phi.reshape(-1), tol,
                 maxit, nthreads, C.byref(E), _ptr(D), npairs, _ptr(out["i"]), _ptr(out["j"]),
                 _ptr(out["e"]), _ptr(out["iters"]), _ptr(out["converged"]), _ptr(out["relres"]))
    if rc < 0:
        raise ValueError(f"o_exx failed ({rc})")
    return E.value, D, out


def solve_pairs(n, cell, r_pe, r_me, centers, phi_by_orbital: dict, pi: Sequence[int], pj: Sequence[int],
                tol=1e-10, maxit=100000, nthreads=0):
    """Solve an explicit pair list; phi_by_orbital maps orbital -> grid array."""
    L = lib()
    Cc = np.ascontiguousarray(centers, np.float64)
    n_orb = Cc.shape[0]
    keep = {k: np.ascontiguousarray(v, np.float64) for k, v in phi_by_orbital.items()}
    ptrs = (C.c_void_p * n_orb)()
    for k, v in keep.items():
        ptrs[k] = v.ctypes.data
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    m = len(pi)
    e, it, cv, rr = np.zeros(m), np.zeros(m, np.int32), np.zeros(m, np.int32), np.zeros(m)
    rpe = np.ascontiguousarray(np.broadcast_to(np.asarray(r_pe, np.float64), (2,)))
    rme = np.ascontiguousarray(np.broadcast_to(np.asarray(r_me, np.float64), (2,)))
    used = L.o_solve_pairs(_i3(n), _d3(cell), rpe, rme, Cc.ravel(), ptrs, m, pi, pj, tol, maxit, nthreads,
                           e, it, cv, rr)
    if used < 0:
        raise ValueError("o_solve_pairs failed")
    return dict(e=e, iters=it, converged=cv, relres=rr, threads=used)


def _phi_table(centers, phi_by_orbital):
    Cc = np.ascontiguousarray(centers, np.float64)
    keep = {k: np.ascontiguousarray(v, np.float64) for k, v in phi_by_orbital.items()}
    ptrs = (C.c_void_p * Cc.shape[0])()
    for k, v in keep.items():
        ptrs[k] = v.ctypes.data
    return Cc, keep, ptrs


def solve_pairs_classed(n, cell, classes, centers, phi_by_orbital: dict, pi, pj, cls, tol=1e-10, maxit=100000,
                        nthreads=0):
    """Solve an explicit pair list with each pair on its own subdomain class:
    classes = [(r_pe, r_me), ...], cls[t] the class of pair t (the per-pair
    subdomains of Sec. IV A)."""
    L = lib()
    Cc, keep, ptrs = _phi_table(centers, phi_by_orbital)
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    cls = np.ascontiguousarray(cls, np.int32)
    m = len(pi)
    rpe = np.ascontiguousarray([c[0] for c in classes], np.float64)
    rme = np.ascontiguousarray([c[1] for c in classes], np.float64)
    e, it, cv, rr = np.zeros(m), np.zeros(m, np.int32), np.zeros(m, np.int32), np.zeros(m)
    used = L.o_solve_pairs_classed(_i3(n), _d3(cell), len(classes), rpe, rme, Cc.ravel(), ptrs, m, pi, pj, cls, tol,
                                   maxit, nthreads, e, it, cv, rr)
    if used < 0:
        raise ValueError("o_solve_pairs_classed failed")
    return dict(e=e, iters=it, converged=cv, relres=rr, threads=used)


def dxx_orbital(n, cell, classes, centers, phi_by_orbital: dict, pi, pj, cls, k, tol=1e-10, maxit=100000,
                nthreads=0):
    """D^k (Eq. Dxx_mlwf_omega) on the full grid from an explicit list of the
    pairs involving orbital k (each on class cls[t]), summed in list order."""
    L = lib()
    Cc, keep, ptrs = _phi_table(centers, phi_by_orbital)
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    cls = np.ascontiguousarray(cls, np.int32)
    rpe = np.ascontiguousarray([c[0] for c in classes], np.float64)
    rme = np.ascontiguousarray([c[1] for c in classes], np.float64)
    Dk = np.zeros(tuple(int(v) for v in reversed(list(n))))
    rc = L.o_dxx_orbital(_i3(n), _d3(cell), len(classes), rpe, rme, Cc.ravel(), ptrs, len(pi), pi, pj, cls, int(k),
                         tol, maxit, nthreads, Dk.reshape(-1))
    if rc != 0:
        raise ValueError("o_dxx_orbital failed")
    return Dk


# ---------------------------------------------------------------------------
# Per-pair subdomains from spreads (the domains Omega_i and Omega_ij that the
# paper outlines for its next version, Sec. IV A).  Readings: Omega_i is the
# ball of radius omega_scale * spread_i about C_i; the PE sphere of a pair,
# centred at its origin g, has to hold Omega_ij = Omega_i cap Omega_j, which
# is taken to need |g - c| + rho for the smallest ball (c, rho) enclosing the
# lens; the pair runs on the smallest of a few fixed radius classes that is
# at least that large (the largest when none is).
# ---------------------------------------------------------------------------

def lens_enclosing_ball(ci, cj, Ri, Rj, cell):
    """Smallest ball enclosing B(C_i, R_i) cap B(C_j, R_j), the centres taken
    under the minimum image.  Returns (f, rho): the ball is centred at
    C_i + f (C_j - C_i) (f in [0, 1]) with radius rho; None when the
    intersection is empty (d >= R_i + R_j).

    With d = |C_j - C_i| and x = (d^2 + R_i^2 - R_j^2) / (2 d) the signed
    distance from C_i to the plane of the two spheres' intersection circle:
    if x <= 0 the intersection holds a great circle of B_i, so B_i itself is
    the smallest enclosing ball; if x >= d the same holds for B_j; otherwise
    both caps are at most hemispheres and the ball on the circle (centre on
    the plane, radius sqrt(R_i^2 - x^2)) holds both.
    """
    dd = min_image_d2(ci, cj, cell)
    d = math.sqrt(dd)
    Ri, Rj = float(Ri), float(Rj)
    if d >= Ri + Rj:
        return None
    if d == 0.0:
        return 0.0, min(Ri, Rj)
    x = (dd + Ri * Ri - Rj * Rj) / (2.0 * d)
    if x <= 0.0:
        return 0.0, Ri
    if x >= d:
        return 1.0, Rj
    return x / d, math.sqrt(Ri * Ri - x * x)


def pair_domain_radius(ci, cj, Ri, Rj, g, cell, n, self_pair):
    """PE radius about the grid point g (pair origin) that holds Omega_ij:
    |g - c| + rho (Omega_ii = Omega_i for the self pair); 0 when empty."""
    if self_pair:
        f, rho = 0.0, float(Ri)
    else:
        ball = lens_enclosing_ball(ci, cj, Ri, Rj, cell)
        if ball is None:
            return 0.0
        f, rho = ball
    e2 = 0.0
    for a in range(3):
        L = float(cell[a])
        h = L / float(n[a])
        d = float(cj[a]) - float(ci[a])
        d -= L * float(_nint(d / L))
        w = float(g[a]) * h - float(ci[a])
        w -= L * float(_nint(w / L))
        u = w - f * d
        e2 += u * u
    return math.sqrt(e2) + rho


def pair_classes(centers, spreads, cell, n, r_pair, omega_scale, class_r_pe):
    """Class of each pair of pair_list(): the smallest k with
    class_r_pe[k] >= pair_domain_radius (the last class otherwise).
    Returns (classes, capped)."""
    Cc = np.asarray(centers, np.float64)
    pi, pj = pair_list(Cc, cell, r_pair)
    out = np.zeros(len(pi), np.int32)
    capped = 0
    for p, (i, j) in enumerate(zip(pi.tolist(), pj.tolist())):
        g = pair_origin(Cc[i], Cc[j], cell, n)
        r = pair_domain_radius(Cc[i], Cc[j], omega_scale * spreads[i], omega_scale * spreads[j], g, cell, n, i == j)
        k = 0
        while k < len(class_r_pe) and class_r_pe[k] < r:
            k += 1
        if k == len(class_r_pe):
            k = len(class_r_pe) - 1
            capped += 1
        out[p] = k
    return out, capped


def exx_classed(n, cell, r_pair, classes, pair_class, centers, phi, tol=1e-10):
    """E_xx and D (Eqs. exx_omega, Dxx_mlwf_omega) with each pair on its own
    subdomain class: classes = [(r_pe, r_me), ...], pair_class[p] for the
    pairs of pair_list().  Each pair is solved by the class's Subdomain; its
    potential v (PE then shell, Alg. 2 order) adds v phi_j to D^i and v phi_i
    to D^j at the grid points (g + offset) mod N."""
    Cc = np.asarray(centers, np.float64)
    phi = np.asarray(phi, np.float64)
    N = np.asarray(n)
    pi, pj = pair_list(Cc, cell, r_pair)
    subs = [Subdomain(n, cell, a, b) for a, b in classes]
    offs = [s.offsets() for s in subs]
    D = np.zeros_like(phi)
    e = np.zeros(len(pi))
    E = 0.0
    for p, (i, j) in enumerate(zip(pi.tolist(), pj.tolist())):
        k = int(pair_class[p])
        g = pair_origin(Cc[i], Cc[j], cell, n)
        r = subs[k].solve_pair(phi[i], phi[j], g, tol=tol)
        e[p] = r["e"]
        E -= (1.0 if i == j else 2.0) * r["e"]
        v = np.concatenate([r["x"], r["vsh"]])
        gx = np.mod(g[None, :] + offs[k], N)
        flat = (gx[:, 2] * N[1] + gx[:, 1]) * N[0] + gx[:, 0]
        Di, Dj = D[i].reshape(-1), D[j].reshape(-1)
        fi, fj = phi[i].reshape(-1), phi[j].reshape(-1)
        np.add.at(Di, flat, v * fj[flat])
        if i != j:
            np.add.at(Dj, flat, v * fi[flat])
    return E, D, dict(i=pi, j=pj, e=e)
