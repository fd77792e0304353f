"""The orbital spreads that feed the per-pair subdomains: for orbitals with no
polynomial correction, synth.spreads equals the root of the second moment of
|phi|^2 about the centre, measured on the generated grid values (s and p
orbitals, several exponents, a centre off the grid and one across the cell
boundary)."""
import numpy as np
import pytest

from paper_1911_10630_amd import synth as S


def _grid_spread(wl, k):
    phi = S.orbital_values_np(wl.orbitals, k, wl.n_grid, wl.cell)
    h = [wl.cell[a] / wl.n_grid[a] for a in range(3)]
    c = wl.orbitals.centers[k]
    d = []
    for a in range(3):
        x = np.arange(wl.n_grid[a]) * h[a] - c[a]
        d.append(x - wl.cell[a] * np.round(x / wl.cell[a]))      # minimum image
    dz, dy, dx = d[2][:, None, None], d[1][None, :, None], d[0][None, None, :]
    w = phi * phi
    return float(np.sqrt(np.sum(w * (dx * dx + dy * dy + dz * dz)) / np.sum(w)))


@pytest.mark.parametrize("kind,alpha", [(0, 0.8), (0, 2.0), (1, 0.8), (1, 1.4)])
def test_spread_is_the_second_moment_of_the_density(kind, alpha):
    cell = (16.0, 16.0, 16.0)
    wl = S.custom((96, 96, 96), cell, [[5.03, 7.91, 8.27], [15.6, 0.3, 8.0]],
                  kind=[kind, kind], alpha=[alpha, alpha], u=[[0.6, 0.0, 0.8], [0.0, 1.0, 0.0]])
    sp = S.spreads(wl.orbitals)
    for k in range(2):
        assert abs(_grid_spread(wl, k) - sp[k]) <= 1e-6 * sp[k]
