"""The FP64 reference gradient (torch float64 autograd over a brute-force pair
list) pinned against central finite differences of the C oracle's loss and
against the exact invariances of L = sum |a|^2 (CPU only)."""
import numpy as np
import pytest

import oracle
from oracle import adjoint_ref
from paper_2606_23891_amd import inputs


def _set(ns=8, seed=9):
    rng = np.random.default_rng(seed)
    f = inputs.lattice_set(ns, seed=seed, jitter=0.25, velocity="gresho", switches=True)
    n = f["x"].shape[0]
    f["h"] = (f["h"] * rng.uniform(0.85, 1.2, n)).astype(np.float32)
    f["mass"] = (f["mass"] * rng.uniform(0.7, 1.3, n)).astype(np.float32)
    f["v"] = (f["v"] + rng.normal(0, 0.3, (n, 3))).astype(np.float32)
    atilde = rng.uniform(0.05, 1.5, n)
    return f, atilde


def test_reference_loss_matches_oracle_forward():
    f, at = _set()
    L, a, gx, gv, gm = adjoint_ref.reference_gradient(f, at)
    d = oracle.density(f["x"], f["mass"], f["h"])
    z = np.zeros(f["x"].shape[0])
    fo = oracle.force(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"], d["rho_dh"], z, np.zeros((z.size, 3)),
                      f["alpha_v"], f["alpha_d"], atilde=at)
    np.testing.assert_allclose(a, fo["a"], rtol=1e-10, atol=1e-10 * np.abs(fo["a"]).max())
    assert L == pytest.approx((fo["a"] ** 2).sum(), rel=1e-12)


def test_reference_gradient_matches_finite_differences():
    f, at = _set()
    _, _, gx, gv, gm = adjoint_ref.reference_gradient(f, at)
    rng = np.random.default_rng(4)
    n = f["x"].shape[0]
    coords = [("x", int(k), int(c)) for k, c in zip(rng.integers(0, n, 8), rng.integers(0, 3, 8))]
    coords += [("v", int(k), int(c)) for k, c in zip(rng.integers(0, n, 4), rng.integers(0, 3, 4))]
    coords += [("m", int(k), 0) for k in rng.integers(0, n, 4)]
    fd = adjoint_ref.fd_gradient(f, at, coords)
    ref = np.array([{"x": gx, "v": gv}[k][i, c] if k != "m" else gm[i] for k, i, c in coords])
    scale = {"x": np.sqrt((gx ** 2).mean()), "v": np.sqrt((gv ** 2).mean()), "m": np.sqrt((gm ** 2).mean())}
    for (k, i, c), a, b in zip(coords, fd, ref):
        assert abs(a - b) <= 1e-5 * max(abs(b), 1e-3 * scale[k]), (k, i, c, a, b)


def test_reference_gradient_invariances():
    f, at = _set()
    _, _, gx, gv, gm = adjoint_ref.reference_gradient(f, at)
    m = f["mass"].astype(np.float64)
    assert np.all(np.abs(gx.sum(0)) <= 1e-10 * np.abs(gx).sum(0))            # translation
    assert np.all(np.abs(gv.sum(0)) <= 1e-10 * np.abs(gv).sum(0))            # Galilean boost
    assert abs((m * gm).sum()) <= 1e-10 * np.abs(m * gm).sum()               # mass scaling
