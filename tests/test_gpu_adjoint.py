"""Hand-written adjoint kernels (through the C-ABI and the autograd Function)
against FP64 central finite differences of the oracle's loss on 64 sampled
coordinates and against the FP64 torch reference gradient, on the 32^3
jittered Gresho lattice (8^3 cells of 64: one tile per cell, each tile's
neighbour walk shared by four waves), and against the reference gradient
alone on 4^3 cells of 512 (eight tiles per cell) and 16^3 cells of 8 (tiles of
8 particles, one wave per tile).

e = |g - g_ref| / max(|g_ref|, 1e-3 * rms(g_ref over that input kind)) <= 1e-4.
The kernels compute in FP64 (components small against their kind's rms are
sums of nearly cancelling pair terms); v.grad and m.grad come back in the
float32 of v and m, one rounding of the final value.  The norm-wise error is
logged beside it."""
import numpy as np
import pytest

import oracle
from oracle import adjoint_ref
from paper_2606_23891_amd import inputs, sph

from gpuhelp import log

pytestmark = pytest.mark.gpu
TOL = 1e-4
FLOOR = 1e-3


def _setup(n_side=32, grid=None):
    ps = inputs.make_config(4, n_side=n_side, grid=grid)
    f = ps.fields
    d = oracle.density(f["x"], f["mass"], f["h"])
    g = oracle.gradient(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"])
    atilde = oracle.balsara(f["h"], f["u"], d["rho"], g["div_v"], g["rot_v"], f["alpha_v"]).astype(np.float32)
    return ps, atilde


def _gpu_grad(ps, atilde):
    import torch

    from paper_2606_23891_amd import autograd

    f = ps.fields
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    dev = "cuda"
    T = lambda a, dt: torch.tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    ctx = autograd.make_context(plan, T(f["h"], torch.float32), T(f["u"], torch.float32),
                                T(atilde, torch.float32), T(f["alpha_d"], torch.float32))
    x = T(f["x"], torch.float64).requires_grad_(True)
    v = T(f["v"], torch.float32).requires_grad_(True)
    m = T(f["mass"], torch.float32).requires_grad_(True)
    a = autograd.acceleration(x, v, m, ctx)
    L = (a.double() ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    out = (float(L.detach()), a.detach().cpu().numpy(), x.grad.cpu().numpy(), v.grad.cpu().numpy(), m.grad.cpu().numpy())
    plan.close()
    return out


def _err(g, ref, scale, floor=FLOOR):
    return np.abs(g - ref) / np.maximum(np.abs(ref), floor * scale)


def test_adjoint_against_reference_and_fd():
    ps, atilde = _setup()
    f = ps.fields
    log(f"adjoint n={ps.n}")
    L, a, gx, gv, gm = _gpu_grad(ps, atilde)
    Lr, ar, rx, rv, rm = adjoint_ref.reference_gradient(f, atilde.astype(np.float64))
    log(f"loss gpu {L:.8e} ref {Lr:.8e}")
    assert L == pytest.approx(Lr, rel=1e-4)
    sc = {k: float(np.sqrt((r ** 2).mean())) for k, r in (("x", rx), ("v", rv), ("m", rm))}
    ex = _err(gx, rx, sc["x"]).max()
    ev = _err(gv, rv, sc["v"]).max()
    em = _err(gm, rm, sc["m"]).max()
    log(f"vs reference gradient: x {ex:.2e} v {ev:.2e} m {em:.2e}")
    for k, g_, r_ in (("x", gx, rx), ("v", gv, rv), ("m", gm, rm)):
        log(f"  {k}: normwise {np.linalg.norm(g_ - r_) / np.linalg.norm(r_):.2e}, "
            f"at floor 1e-6 max {_err(g_, r_, sc[k], 1e-6).max():.2e}")
    assert max(ex, ev, em) <= TOL, (ex, ev, em)
    # 64 coordinates: 32 positions, 16 velocities, 16 masses (seed 4)
    rng = np.random.default_rng(4)
    n = ps.n
    coords = []
    for kind, want in (("x", 32), ("v", 16), ("m", 16)):
        while sum(1 for c in coords if c[0] == kind) < want:
            c = (kind, int(rng.integers(0, n)), int(rng.integers(0, 3)) if kind != "m" else 0)
            if adjoint_ref.straddles_kink(f, *c):   # resample coordinates on the viscosity kink
                log(f"resampled {c}: its step crosses v_ij . r_ij = 0")
                continue
            coords.append(c)
    fd = adjoint_ref.fd_gradient(f, atilde.astype(np.float64), coords)
    worst = 0.0
    for (kind, k, c), fdv in zip(coords, fd):
        g = {"x": gx[k, c], "v": gv[k, c], "m": gm[k]}[kind]
        e = abs(g - fdv) / max(abs(fdv), FLOOR * sc[kind])
        worst = max(worst, e)
        assert e <= TOL, (kind, k, c, g, fdv, e)
    log(f"vs finite differences: worst {worst:.2e}")
    # exact invariances of L hold for the adjoint up to rounding (v.grad and
    # m.grad carry the float32 rounding of v and m)
    m = f["mass"].astype(np.float64)
    assert np.all(np.abs(gx.sum(0)) <= 1e-10 * np.abs(gx).sum(0))
    assert np.all(np.abs(gv.sum(0)) <= 1e-6 * np.abs(gv).sum(0))
    assert abs((m * gm).sum()) <= 1e-6 * np.abs(m * gm).sum()


@pytest.mark.parametrize("grid", [4, 16])
def test_adjoint_cell_grids(grid):
    ps, atilde = _setup(grid=grid)
    f = ps.fields
    log(f"adjoint n={ps.n} grid {grid}^3: {inputs.cell_stats(ps.cells)}")
    L, a, gx, gv, gm = _gpu_grad(ps, atilde)
    Lr, ar, rx, rv, rm = adjoint_ref.reference_gradient(f, atilde.astype(np.float64))
    assert L == pytest.approx(Lr, rel=1e-4)
    ea = _err(a, ar, float(np.sqrt((ar ** 2).mean()))).max()
    sc = {k: float(np.sqrt((r ** 2).mean())) for k, r in (("x", rx), ("v", rv), ("m", rm))}
    ex = _err(gx, rx, sc["x"]).max()
    ev = _err(gv, rv, sc["v"]).max()
    em = _err(gm, rm, sc["m"]).max()
    log(f"grid {grid}: a {ea:.2e}; gradient x {ex:.2e} v {ev:.2e} m {em:.2e}")
    assert max(ea, ex, ev, em) <= TOL, (ea, ex, ev, em)
