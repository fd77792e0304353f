"""Seeded synthetic workloads: localized orbitals on a periodic grid.

This module only draws and evaluates *inputs*.  It contains none of the
exchange method's arithmetic (no pair list, no Poisson solve, no
multipoles); both the CPU oracle tests and the GPU path consume the arrays
it produces.

Units are Hartree atomic units (bohr) throughout, as in the paper's
Poisson equation (Sec. II.C, Eq. pe).  Workload sizes are quoted in
angstrom and converted with the CODATA-2018 bohr radius.

Orbital recipe (every workload)
-------------------------------
* type s or p with probability 1/2;
  s: exp(-alpha |d|^2),  p: (u . d) exp(-alpha |d|^2), u a random unit vector;
* multiplied by P(d) = 1 + a.d + d^T B d, a_k ~ U[-0.3, 0.3] /bohr,
  symmetric B_kl ~ U[-0.1, 0.1] /bohr^2;
* alpha ~ U[0.8, 2.0] /bohr^2;
* d = r - C under the minimum-image convention of the orthorhombic cell;
* normalized on the grid: h_x h_y h_z sum(phi^2) = 1.

These stand in for the maximally localized Wannier functions of liquid
water used by the paper (Sec. IV), which are not available here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

BOHR_ANGSTROM = 0.529177210903          # CODATA 2018, angstrom per bohr
ANG = 1.0 / BOHR_ANGSTROM               # bohr per angstrom


@dataclasses.dataclass
class OrbitalSet:
    """Seeded description of n_orb orbitals (parameters, not grid values)."""
    centers: np.ndarray      # [n, 3] bohr, inside [0, L)
    kind: np.ndarray         # [n] 0 = s, 1 = p
    alpha: np.ndarray        # [n] bohr^-2
    u: np.ndarray            # [n, 3] unit vectors (p type)
    a: np.ndarray            # [n, 3] bohr^-1
    B: np.ndarray            # [n, 3, 3] bohr^-2, symmetric

    @property
    def n(self) -> int:
        return int(self.centers.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    n_grid: tuple            # (Nx, Ny, Nz)
    cell: tuple              # (Lx, Ly, Lz) bohr
    orbitals: OrbitalSet
    r_pair: float            # bohr
    r_pe: tuple              # (self, non-self) bohr
    r_me: tuple              # (self, non-self) bohr
    cg_rtol: float = 1e-10
    orbital_dtype: str = "f64"
    precision: str = "fp64"  # "fp64" | "fp32_refine"
    md_steps: int = 1
    seed: int = 0
    box: Optional[tuple] = None   # orbital storage box (bx, by, bz); None = whole grid

    @property
    def h(self) -> tuple:
        return tuple(self.cell[a] / self.n_grid[a] for a in range(3))


def _random_unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def draw_orbital_shapes(rng, centers: np.ndarray) -> OrbitalSet:
    n = centers.shape[0]
    kind = (rng.random(n) < 0.5).astype(np.int32)
    alpha = rng.uniform(0.8, 2.0, size=n)
    u = _random_unit(rng, n)
    a = rng.uniform(-0.3, 0.3, size=(n, 3))
    Bu = rng.uniform(-0.1, 0.1, size=(n, 3, 3))
    B = 0.5 * (Bu + np.transpose(Bu, (0, 2, 1)))
    return OrbitalSet(centers=np.ascontiguousarray(centers, dtype=np.float64),
                      kind=kind, alpha=alpha, u=u, a=a, B=B)


def _min_image_1d(coord: np.ndarray, c: float, L: float) -> np.ndarray:
    d = coord - c
    return d - L * np.round(d / L)


def orbital_values_np(orbs: OrbitalSet, k: int, n_grid, cell, origin=(0, 0, 0), box=None) -> np.ndarray:
    """Values of orbital k, numpy float64, layout [Nz][Ny][Nx]; or, with a
    box (bx, by, bz) starting at grid point `origin`, on that periodic box
    [bz][by][bx], normalized on the box (the orbital is zero outside it)."""
    Nx, Ny, Nz = n_grid
    bx, by, bz = box if box is not None else (Nx, Ny, Nz)
    h = [cell[a] / n_grid[a] for a in range(3)]
    c = orbs.centers[k]
    dx = _min_image_1d(((origin[0] + np.arange(bx)) % Nx) * h[0], c[0], cell[0])[None, None, :]
    dy = _min_image_1d(((origin[1] + np.arange(by)) % Ny) * h[1], c[1], cell[1])[None, :, None]
    dz = _min_image_1d(((origin[2] + np.arange(bz)) % Nz) * h[2], c[2], cell[2])[:, None, None]
    al = orbs.alpha[k]
    g = np.exp(-al * dx * dx) * np.exp(-al * dy * dy) * np.exp(-al * dz * dz)
    if orbs.kind[k] == 1:
        u = orbs.u[k]
        g = g * (u[0] * dx + u[1] * dy + u[2] * dz)
    a = orbs.a[k]
    B = orbs.B[k]
    P = (1.0 + a[0] * dx + a[1] * dy + a[2] * dz
         + B[0, 0] * dx * dx + B[1, 1] * dy * dy + B[2, 2] * dz * dz
         + 2.0 * (B[0, 1] * dx * dy + B[0, 2] * dx * dz + B[1, 2] * dy * dz))
    phi = g * P
    nrm = math.sqrt(h[0] * h[1] * h[2] * float(np.sum(phi * phi)))
    return phi / nrm


def orbitals_np(wl: Workload, idx: Optional[Sequence[int]] = None, origins=None) -> np.ndarray:
    """All (or selected) orbitals as numpy float64 [n][Nz][Ny][Nx], or on the
    workload's boxes [n][bz][by][bx] given the box origins [n_orb][3]."""
    idx = range(wl.orbitals.n) if idx is None else idx
    box = wl.box if origins is not None else None
    bx, by, bz = box if box is not None else wl.n_grid
    out = np.empty((len(idx), bz, by, bx), dtype=np.float64)
    for o, k in enumerate(idx):
        org = tuple(origins[k]) if origins is not None else (0, 0, 0)
        out[o] = orbital_values_np(wl.orbitals, k, wl.n_grid, wl.cell, org, box)
    return out


def embed_boxes(vals: np.ndarray, origins, n_grid) -> np.ndarray:
    """Box arrays [n][bz][by][bx] placed (periodically) into zero grids [n][Nz][Ny][Nx]."""
    Nx, Ny, Nz = n_grid
    n, bz, by, bx = vals.shape
    out = np.zeros((n, Nz, Ny, Nx), dtype=vals.dtype)
    for k in range(n):
        ox, oy, oz = (int(v) for v in origins[k])
        ix = (ox + np.arange(bx)) % Nx
        iy = (oy + np.arange(by)) % Ny
        iz = (oz + np.arange(bz)) % Nz
        out[k][np.ix_(iz, iy, ix)] = vals[k]
    return out


def extract_boxes(full: np.ndarray, origins, box) -> np.ndarray:
    """The inverse of embed_boxes: box arrays cut (periodically) from grids."""
    n, Nz, Ny, Nx = full.shape
    bx, by, bz = box
    out = np.empty((n, bz, by, bx), dtype=full.dtype)
    for k in range(n):
        ox, oy, oz = (int(v) for v in origins[k])
        out[k] = full[k][np.ix_((oz + np.arange(bz)) % Nz, (oy + np.arange(by)) % Ny, (ox + np.arange(bx)) % Nx)]
    return out


def orbitals_torch(wl: Workload, device="cpu", dtype=None, origins=None, out=None):
    """All orbitals as a torch tensor [n][Nz][Ny][Nx] on `device`, or on the
    workload's boxes [n][bz][by][bx] given the box origins [n_orb][3];
    written into `out` when given.

    Values are evaluated in float64 with the same formula as
    :func:`orbital_values_np` and cast to `dtype` at the end.
    """
    import torch
    f64 = torch.float64
    dtype = dtype or (torch.float64 if wl.orbital_dtype == "f64" else torch.float32)
    orbs = wl.orbitals
    Nx, Ny, Nz = wl.n_grid
    bx, by, bz = wl.box if origins is not None else (Nx, Ny, Nz)
    h = wl.h
    if out is None:
        out = torch.empty((orbs.n, bz, by, bx), dtype=dtype, device=device)

    def mi(coord, c, L):
        d = coord - c
        return d - L * torch.round(d / L)

    def axis(o, b, N, hh):
        return ((o + torch.arange(b, device=device)) % N).to(f64) * hh

    for k in range(orbs.n):
        c = orbs.centers[k]
        o = origins[k] if origins is not None else (0, 0, 0)
        dx = mi(axis(int(o[0]), bx, Nx, h[0]), float(c[0]), wl.cell[0]).view(1, 1, bx)
        dy = mi(axis(int(o[1]), by, Ny, h[1]), float(c[1]), wl.cell[1]).view(1, by, 1)
        dz = mi(axis(int(o[2]), bz, Nz, h[2]), float(c[2]), wl.cell[2]).view(bz, 1, 1)
        al = float(orbs.alpha[k])
        g = torch.exp(-al * dx * dx) * torch.exp(-al * dy * dy) * torch.exp(-al * dz * dz)
        if orbs.kind[k] == 1:
            u = orbs.u[k]
            g = g * (float(u[0]) * dx + float(u[1]) * dy + float(u[2]) * dz)
        a = orbs.a[k]
        B = orbs.B[k]
        P = (1.0 + float(a[0]) * dx + float(a[1]) * dy + float(a[2]) * dz
             + float(B[0, 0]) * dx * dx + float(B[1, 1]) * dy * dy + float(B[2, 2]) * dz * dz
             + 2.0 * (float(B[0, 1]) * dx * dy + float(B[0, 2]) * dx * dz
                      + float(B[1, 2]) * dy * dz))
        phi = g * P
        nrm = math.sqrt(h[0] * h[1] * h[2] * float(torch.sum(phi * phi)))
        out[k] = (phi / nrm).to(dtype)
    return out


# ---------------------------------------------------------------------------
# Centre layouts
# ---------------------------------------------------------------------------

def _random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


_TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) / math.sqrt(3.0)


def water_centers(rng, n_side: int, L: float, bcc: bool) -> np.ndarray:
    """Four orbital centres per molecule, 0.5 A from a jittered-lattice O."""
    a = L / n_side
    sites = [(i, j, k) for k in range(n_side) for j in range(n_side) for i in range(n_side)]
    O = [np.array(s, dtype=np.float64) * a for s in sites]
    if bcc:
        O += [(np.array(s, dtype=np.float64) + 0.5) * a for s in sites]
    O = np.array(O)
    O = O + rng.uniform(-0.25 * ANG, 0.25 * ANG, size=O.shape)
    cen = []
    for o in O:
        R = _random_rotation(rng)
        for t in _TETRA:
            cen.append(o + 0.5 * ANG * (R @ t))
    cen = np.array(cen)
    return np.mod(cen, L)


def _min_image_dists(C: np.ndarray, L: float) -> np.ndarray:
    d = C[None, :, :] - C[:, None, :]
    d -= L * np.round(d / L)
    return np.sqrt(np.sum(d * d, axis=-1))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def c1_small(seed: int = 1234) -> Workload:
    """16 orbitals in a 10 A cube, 48^3 grid, ~60 pairs, FP64."""
    L = 10.0 * ANG
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, L, size=(16, 3))
    orbs = draw_orbital_shapes(rng, C)
    d = _min_image_dists(C, L)
    iu = np.triu_indices(16, k=1)
    ds = np.sort(d[iu])
    r_pair = 0.5 * (ds[43] + ds[44])     # 16 self + 44 non-self = 60 pairs
    return Workload("small-16orb-48^3", (48, 48, 48), (L, L, L), orbs, float(r_pair),
                    (4.0 * ANG, 4.0 * ANG), (5.0 * ANG, 5.0 * ANG), seed=seed)


def _water(name, n_side, L_ang, N, bcc, seed, **kw) -> Workload:
    L = L_ang * ANG
    rng = np.random.default_rng(seed)
    C = water_centers(rng, n_side, L, bcc)
    orbs = draw_orbital_shapes(rng, C)
    r_pe = kw.pop("r_pe", (4.0 * ANG, 4.0 * ANG))
    r_me = kw.pop("r_me", (5.0 * ANG, 5.0 * ANG))
    return Workload(name, (N, N, N), (L, L, L), orbs, kw.pop("r_pair", 5.0 * ANG),
                    r_pe, r_me, seed=seed, **kw)


def c2_water64(seed: int = 64) -> Workload:
    """64 H2O (256 orbitals), 12.4 A cube, 128^3 grid, R_pair 5 A, FP64."""
    return _water("water64-128^3-fp64", 4, 12.4, 128, False, seed)


def c3_water64_mixed(seed: int = 64) -> Workload:
    """Same system as c2; stencil-CG in FP32 with FP64 refinement."""
    return _water("water64-128^3-fp32refine", 4, 12.4, 128, False, seed, precision="fp32_refine")


def c4_water128(seed: int = 128) -> Workload:
    """128 H2O (512 orbitals), 15.6 A cube, 160^3 grid, 10-step MD."""
    return _water("water128-160^3", 4, 15.6, 160, True, seed, md_steps=10)


def c5_water512(seed: int = 512) -> Workload:
    """512 H2O (2048 orbitals), 24.8 A cube, 256^3, FP32 orbitals on 160^3
    local boxes, two subdomain classes."""
    rpe_ns = 4.0 * ANG * 5.0 / 6.0
    return _water("water512-256^3-uneven", 8, 24.8, 256, False, seed,
                  r_pe=(4.0 * ANG, rpe_ns), r_me=(5.0 * ANG, rpe_ns + 1.0 * ANG),
                  orbital_dtype="f32", precision="fp32_refine", md_steps=5, box=(160, 160, 160))


def c1_boxed(seed: int = 4321) -> Workload:
    """16 orbitals in a 20 A cube (96^3 grid, the small workload's spacing),
    R_pair 4.5 A, stored on 76^3 local boxes: the small-scale check of
    box storage."""
    L = 20.0 * ANG
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, L, size=(16, 3))
    orbs = draw_orbital_shapes(rng, C)
    return Workload("boxed16-96^3", (96, 96, 96), (L, L, L), orbs, 4.5 * ANG, (4.0 * ANG, 4.0 * ANG),
                    (5.0 * ANG, 5.0 * ANG), seed=seed, box=(76, 76, 76))


def spreads(orbs: OrbitalSet) -> np.ndarray:
    """Spread of each orbital (bohr): the root of the second moment of |phi|^2
    about the centre for the Gaussian factor, 3 / (4 alpha) for s and
    5 / (4 alpha) for p orbitals (the small polynomial corrections ignored)."""
    m2 = np.where(orbs.kind == 1, 5.0, 3.0) / (4.0 * orbs.alpha)
    return np.sqrt(m2)


def md_displace(orbs: OrbitalSet, L: float, rng, sigma_ang: float = 0.02) -> OrbitalSet:
    """One synthetic MD step: Gaussian centre displacement, shapes fixed."""
    C = np.mod(orbs.centers + rng.normal(scale=sigma_ang * ANG, size=orbs.centers.shape), L)
    return dataclasses.replace(orbs, centers=C)


def custom(n_grid, cell, centers, kind=None, alpha=None, u=None, a=None, B=None,
           r_pair=5.0 * ANG, r_pe=4.0 * ANG, r_me=5.0 * ANG, name="custom") -> Workload:
    """Hand-built workload (tests): unspecified shape parameters default to a
    plain s Gaussian with alpha = 1 and no polynomial factor."""
    C = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    n = C.shape[0]
    orbs = OrbitalSet(
        centers=C,
        kind=np.zeros(n, np.int32) if kind is None else np.asarray(kind, np.int32),
        alpha=np.ones(n) if alpha is None else np.asarray(alpha, np.float64),
        u=np.tile([1.0, 0.0, 0.0], (n, 1)) if u is None else np.asarray(u, np.float64),
        a=np.zeros((n, 3)) if a is None else np.asarray(a, np.float64),
        B=np.zeros((n, 3, 3)) if B is None else np.asarray(B, np.float64))
    rpe = r_pe if isinstance(r_pe, tuple) else (r_pe, r_pe)
    rme = r_me if isinstance(r_me, tuple) else (r_me, r_me)
    return Workload(name, tuple(n_grid), tuple(cell), orbs, r_pair, rpe, rme)


WORKLOADS = {
    "c1": c1_small,
    "c2": c2_water64,
    "c3": c3_water64_mixed,
    "c4": c4_water128,
    "c5": c5_water512,
}
