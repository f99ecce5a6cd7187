"""Smoothing-length iteration through the C-ABI against the oracle's.

Both start from the same perturbed float32 h.  The GPU steps in FP32 on FP32
densities, the oracle in FP64, so a particle's last accepted step can differ
by up to the tolerance: final h agree within 3 tol h, and each side's h solves
rho(h) h^3 = m eta^3 to within 5 tol (relative) on the FP64 density.  The
densities left in the store are those of the final h (1e-5 on the oracle's
tolerance scale)."""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

from gpuhelp import compare_loop, device_store, log, outputs

pytestmark = pytest.mark.gpu
ETA, TOL = 1.2348, 1e-4


def _perturbed(ps, seed):
    rng = np.random.default_rng(seed)
    h = (ps.fields["h"] * rng.uniform(0.8, 1.25, ps.n)).astype(np.float32)
    return h


def _reach(ps):
    """the oracle's reach of every particle's cell (the support its tasks cover)"""
    return oracle.particle_reach(ps.cells, ps.tasks, ps.n)


@pytest.mark.parametrize("name,cfg", [("lattice16", dict(k=0, n_side=16, grid=4)),
                                      ("grid512", dict(k=2, n_side=32, grid=4))])
def test_h_iteration_matches_oracle(name, cfg):
    import torch
    ps = inputs.make_config(cfg["k"], n_side=cfg["n_side"], grid=cfg["grid"])
    h0 = _perturbed(ps, 3)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, sph.LAYOUTS.index("SAOS_SHARED"), extra={"h": h0})
    ws = torch.zeros(sph.sph_h_iterate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    log(f"h iteration {name} n={ps.n}")
    passes, still = sph.sph_h_iterate(plan, st, ws, eta=ETA, tol=TOL, max_iter=30)
    torch.cuda.synchronize()
    hg = st.get("h")
    log(f"{name}: GPU passes {passes}, unconverged {still}")
    ref = oracle.h_iterate(ps.fields["x"], ps.fields["mass"], h0, _reach(ps), eta=ETA, tol=TOL)
    log(f"{name}: oracle passes {ref['passes']}, unconverged {ref['unconverged']}")
    assert still == 0 and ref["unconverged"] == 0
    assert passes >= 2
    hr = ref["h"].astype(np.float64)
    assert np.max(np.abs(hg - hr) / hr) <= 3 * TOL
    m = ps.fields["mass"].astype(np.float64)
    for h in (hg, ref["h"]):
        d = oracle.density(ps.fields["x"], ps.fields["mass"], h)
        res = np.abs(d["rho"] * h.astype(np.float64) ** 3 - m * ETA ** 3) / (m * ETA ** 3)
        assert res.max() <= 5 * TOL, res.max()
    # the store's density outputs belong to its final h
    ref_d = oracle.density(ps.fields["x"], ps.fields["mass"], hg, epsx=oracle.pack_resolution(ps.cells))
    errs = compare_loop(0, outputs(st, 0), ref_d)
    log(f"{name}: density at final h, worst {max(errs.values()):.2e}")
    assert max(errs.values()) <= 1e-5, errs
    plan.close()


def test_h_iteration_pass_limit_and_arguments():
    import torch
    ps = inputs.make_config(0, n_side=16, grid=4)
    h0 = _perturbed(ps, 5)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, sph.LAYOUTS.index("AOS"), extra={"h": h0})
    ws = torch.zeros(sph.sph_h_iterate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    log("h iteration, one pass")
    passes, still = sph.sph_h_iterate(plan, st, ws, eta=ETA, tol=TOL, max_iter=1)
    torch.cuda.synchronize()
    ref = oracle.h_iterate(ps.fields["x"], ps.fields["mass"], h0, _reach(ps), eta=ETA, tol=TOL, max_iter=1)
    assert passes == 1 and still > 0
    # one pass: the first density is of h0 on both sides, so the stepped h agree to FP32 step rounding
    assert np.max(np.abs(st.get("h") - ref["h"]) / ref["h"]) <= 1e-5
    assert abs(still - ref["unconverged"]) <= max(2, ps.n // 1000)
    for bad in (dict(eta=0.0), dict(tol=0.0), dict(max_iter=0)):
        kw = dict(eta=ETA, tol=TOL, max_iter=5)
        kw.update(bad)
        with pytest.raises(sph.SphError):
            sph.sph_h_iterate(plan, st, ws, **kw)
    with pytest.raises(sph.SphError):
        sph.sph_h_iterate(plan, st, ws[:256], eta=ETA, tol=TOL, max_iter=5)
    plan.close()


def test_plan_reach_matches_oracle():
    """the plan's per-cell reach (bucketed search) against the oracle's brute
    force over all cell pairs: a uniform grid (the cell width), the clustered
    set's octree with six cell widths, and a sparse grid with empty cells"""
    for name, ps in (("grid8", inputs.make_config(1, n_side=32, grid=8)),
                     ("octree64", inputs.make_config(3, n_side=64)),
                     ("octree24", inputs.make_config(3, n_side=24))):
        plan = sph.Plan(ps.cells, ps.tasks, ps.n)
        got = plan.cell_reach()
        ref = oracle.cell_reach(ps.cells, ps.tasks)
        log(f"reach {name}: cells {len(ps.cells)}, reach/width {np.min(got / ps.cells['width']):.3f}.."
            f"{np.max(got / ps.cells['width']):.3f}")
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)
        plan.close()


def test_h_iteration_octree_with_cell_caps():
    """the clustered set's octree at 64^3 (cells of six widths, supports
    beyond the smaller cells) with eta = 3: supports of several hundred
    neighbours, so the dense regions reach the cap gamma_K h <= the reach of
    their cell and stay there; GPU and oracle apply the same limits, so the
    final h agree, and the stored densities are those of the final h, checked
    against the oracle's density on every particle"""
    import torch
    ps = inputs.make_config(3, n_side=64)
    eta = 3.0   # supports of several hundred neighbours: the dense regions reach the cap
    h0 = (_perturbed(ps, 7) * np.float32(eta / ETA)).astype(np.float32)
    reach = _reach(ps)
    h0 = np.minimum(h0, (reach / oracle.GAMMA_K).astype(np.float32))
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, sph.LAYOUTS.index("SOA"), extra={"h": h0})
    ws = torch.zeros(sph.sph_h_iterate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    log(f"h iteration octree n={ps.n} cells={len(ps.cells)} widths {np.unique(ps.cells['width']).size}")
    passes, still = sph.sph_h_iterate(plan, st, ws, eta=eta, tol=TOL, max_iter=40)
    torch.cuda.synchronize()
    hg = st.get("h")
    ref = oracle.h_iterate(ps.fields["x"], ps.fields["mass"], h0, reach, eta=eta, tol=TOL, max_iter=40)
    capped = hg.astype(np.float64) * oracle.GAMMA_K >= reach * (1 - 1e-6)
    log(f"octree: GPU passes {passes} left {still}; oracle passes {ref['passes']} left {ref['unconverged']}; "
        f"capped {int(capped.sum())}, in cells narrower than their support "
        f"{int(np.sum(oracle.GAMMA_K * hg > np.repeat(ps.cells['width'], ps.cells['count'])))}")
    assert still == 0 and ref["unconverged"] == 0
    hr = ref["h"].astype(np.float64)
    assert np.max(np.abs(hg - hr) / hr) <= 3 * TOL
    assert capped.sum() > 100
    assert np.all(oracle.GAMMA_K * hg.astype(np.float64) <= reach * (1 + 1e-6))
    ref_d = oracle.density(ps.fields["x"], ps.fields["mass"], hg, epsx=oracle.pack_resolution(ps.cells),
                           grid=True)
    errs = compare_loop(0, outputs(st, 0), ref_d)
    log(f"octree: density at final h, worst {max(errs.values()):.2e}")
    assert max(errs.values()) <= 1e-5, errs
    plan.close()
