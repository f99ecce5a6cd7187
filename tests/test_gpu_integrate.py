"""Time integration around the loops through the C-ABI against the oracle.

Kick, drift, the distance outside the cells and the CFL step are plain
float32 / float64 operations, each rounded once: bit for bit.  A whole
kick-drift-kick step: positions bit for bit, the new accelerations and
heating rates within the force loop's tolerance, and the second half kick
bit for bit given the GPU's own accelerations."""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

from gpuhelp import LOOP_OUT, compare_loop, device_store, log, oracle_loop, outputs

pytestmark = pytest.mark.gpu


def _setup(seed=21, layout="SAOS_SHARED"):
    import torch
    ps = inputs.make_config(0, n_side=16, grid=4)
    f = inputs.random_fields(ps.n, seed, x=ps.fields["x"])
    f["h"] = ps.fields["h"]
    f["v_sig"] = np.abs(f["v_sig"])
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = sph.Store(sph.LAYOUTS.index(layout), ps.n)
    st.put_all(f)
    ws = torch.zeros(sph.sph_integrate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    return ps, f, plan, st, ws


@pytest.mark.parametrize("layout", ["AOS", "SAOS_SHARED", "SOA", "SAOS_SHARED_REPL"])
def test_kick_drift_cfl_bitexact(layout):
    import torch
    ps, f, plan, st, ws = _setup(layout=layout)
    log(f"kick / drift / cfl {layout} n={ps.n}")
    sph.sph_kick(st, 0.0123)
    v, u = oracle.kick(f["v"], f["a"], f["u"], f["u_dt"], 0.0123)
    assert st.get("v").tobytes() == v.tobytes()
    assert st.get("u").tobytes() == u.tobytes()
    mo, mh = sph.sph_drift(plan, st, 0.0371, ws)
    xn, out = oracle.drift(f["x"], v, 0.0371, ps.cells)
    assert st.get("x").tobytes() == xn.tobytes()
    assert mo == out.max()
    assert mh == f["h"].max()
    # the whole store, every copy of a replicated position included, as the
    # oracle's store of the kicked and drifted fields
    host = oracle.HostStore(sph.LAYOUTS.index(layout), ps.n)
    host.put_all(dict(f, v=v, u=u, x=xn))
    assert st.raw() == host.raw()
    dt = sph.sph_cfl_dt(plan, st, ws, cfl=0.2)
    assert np.float32(dt) == oracle.cfl_dt(f["h"], f["v_sig"], 0.2)
    torch.cuda.synchronize()
    plan.close()


def test_kdk_step_matches_oracle():
    import torch
    ps = inputs.make_config(1, n_side=16, grid=4)
    lay = sph.LAYOUTS.index("SAOS_SHARED")
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, lay)
    sws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    sph.sph_step_batched(plan, st, sws)   # a, u_dt and V of the starting state
    iws = torch.zeros(sph.sph_integrate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    dt = sph.sph_cfl_dt(plan, st, iws, cfl=0.1)
    log(f"kdk step n={ps.n} dt={dt:.3e}")
    names = ("x", "v", "a", "mass", "h", "u", "u_dt", "alpha_v", "alpha_d")
    f0 = {k: st.get(k) for k in names}
    ws = torch.zeros(sph.kdk_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    assert sph.sph_step_kdk(plan, st, ws, dt) == 0
    torch.cuda.synchronize()
    half = np.float32(0.5) * np.float32(dt)
    vh, uh = oracle.kick(f0["v"], f0["a"], f0["u"], f0["u_dt"], half)
    xn, _ = oracle.drift(f0["x"], vh, np.float64(np.float32(dt)), ps.cells)
    assert st.get("x").tobytes() == xn.tobytes()
    # the loops at the drifted state, each fed the GPU's previous-loop outputs
    f1 = dict(f0, x=xn, v=vh, u=uh)
    eps = oracle.pack_resolution(ps.cells)
    prev = {}
    for loop in range(3):
        g = outputs(st, loop)
        errs = compare_loop(loop, g, oracle_loop(f1, loop, prev, epsx=eps))
        log(f"kdk step: loop {loop} worst {max(errs.values()):.2e}")
        assert max(errs.values()) <= 1e-5, errs
        for k in LOOP_OUT[loop]:
            prev[k] = g[k].astype(np.float64)
    # the second half kick, given the GPU's accelerations
    v2, u2 = oracle.kick(vh, st.get("a"), uh, st.get("u_dt"), half)
    assert st.get("v").tobytes() == v2.tobytes()
    assert st.get("u").tobytes() == u2.tobytes()
    plan.close()


def test_kdk_stops_when_particles_leave_the_reach():
    import torch
    ps = inputs.make_config(1, n_side=16, grid=4)
    lay = sph.LAYOUTS.index("SOA")
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, lay)
    sws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    sph.sph_step_batched(plan, st, sws)
    f0 = {k: st.get(k) for k in ("x", "v", "a", "u", "u_dt")}
    ws = torch.zeros(sph.kdk_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    log("kdk with a step far beyond the reach")
    with pytest.raises(sph.SphError) as e:
        sph.sph_step_kdk(plan, st, ws, 0.5)
    assert e.value.status == -4   # SPH_E_PLAN
    torch.cuda.synchronize()
    vh, uh = oracle.kick(f0["v"], f0["a"], f0["u"], f0["u_dt"], np.float32(0.25))
    xn, _ = oracle.drift(f0["x"], vh, 0.5, ps.cells)
    assert st.get("x").tobytes() == xn.tobytes()
    assert st.get("v").tobytes() == vh.tobytes()
    plan.close()
