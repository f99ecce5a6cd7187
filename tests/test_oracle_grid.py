"""The oracle's candidate grid against its brute force (CPU only).

With grid=True the loops visit, for each row, the particles of the 27 grid
cells around it in ascending index order instead of every particle; the grid
is only a way of skipping particles that cannot interact.  Every output (sums,
error scales, signal-velocity maxima, pair counts, edge bands) must equal the
brute-force result bit for bit, on the 16^3 lattice (all rows), on sampled rows
of the 32^3 and 64^3 Gresho lattices, and on sampled rows of a clustered set
whose supports span a factor of 100.
"""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs


def _loops(f, rows, eps, grid):
    d = oracle.density(f["x"], f["mass"], f["h"], rows=rows, epsx=eps, grid=grid)
    # the later loops take every particle's previous outputs: use the rows'
    # own values where sampled and a smooth stand-in elsewhere (the same
    # inputs for both modes)
    n = f["x"].shape[0]
    rho = np.full(n, 1.0)
    g = oracle.gradient(f["x"], f["v"], f["mass"], f["h"], f["u"], rho, rows=rows, epsx=eps, grid=grid)
    rng = np.random.default_rng(5)
    D = rng.normal(0, 1e-2, n)
    R = rng.normal(0, 1e-2, (n, 3))
    fo = oracle.force(f["x"], f["v"], f["mass"], f["h"], f["u"], rho, np.full(n, -0.03), D, R,
                      f["alpha_v"], f["alpha_d"], rows=rows, epsx=eps, grid=grid)
    return d, g, fo


def _same(a, b):
    for k in a:
        assert np.asarray(a[k]).tobytes() == np.asarray(b[k]).tobytes(), k


@pytest.mark.parametrize("k,n_side,nrows", [(0, None, None), (4, 32, 3000), (1, 64, 1500), (3, 48, 1500)])
def test_grid_equals_brute_force(k, n_side, nrows):
    ps = inputs.make_config(k, n_side=n_side) if n_side else inputs.make_config(k)
    f = ps.fields
    rows = None if nrows is None else np.sort(np.random.default_rng(9).choice(ps.n, nrows, replace=False))
    eps = oracle.pack_resolution(ps.cells)
    brute = _loops(f, rows, eps, False)
    fast = _loops(f, rows, eps, True)
    for b, q in zip(brute, fast):
        _same(b, q)
    # the grid did take effect (more than 3 cells per side) on the lattices
    if k != 3:
        H = oracle.GAMMA_K * float(np.max(f["h"]))
        assert int(1.0 / (1.0001 * H + 2 * float(np.max(eps)))) >= 3
