"""The batched form as one captured HIP graph, replayed several times with
eager work and synchronisation between replays: every replay must reproduce
the eager step bit for bit (the kernels are deterministic).  Also sparse grids
with empty and single-particle cells."""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

from gpuhelp import LOOP_OUT, compare_loop, device_store, log, oracle_loop, outputs, run_batched_loop, run_per_task

pytestmark = pytest.mark.gpu
OUT_FIELDS = [k for L in range(3) for k in LOOP_OUT[L]]


def _snapshot(st):
    return {k: st.get(k).copy() for k in OUT_FIELDS}


def test_graph_replays_match_eager_step():
    import torch
    ps = inputs.make_config(1, n_side=32)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    st = device_store(ps, sph.LAYOUTS.index("SAOS_SHARED_TYPE"))
    sph.sph_step_batched(plan, st, ws)
    torch.cuda.synchronize()
    ref = _snapshot(st)
    # the step chained from the individual stages gives the same bits
    st2 = device_store(ps, sph.LAYOUTS.index("SAOS_SHARED_TYPE"))
    for L in range(3):
        run_batched_loop(plan, st2, L)
    s2 = _snapshot(st2)
    for k in OUT_FIELDS:
        assert np.array_equal(s2[k], ref[k]), k
    # the fused kernels and a split schedule (several pack / unpack launches
    # per loop inside the graph) replay to the same bits
    for sched in (0, 4):
        tn = sph.default_tuning()
        tn.pack_schedule = sched
        g = sph.Graph(plan, st, ws, tuning=tn)
        for rep in range(4):
            log(f"graph replay {rep} schedule {sched}")
            st.put("rho", np.zeros(ps.n, np.float32))       # eager work between replays
            st.put("a", np.full((ps.n, 3), 7.0, np.float32))
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            got = _snapshot(st)
            for k in OUT_FIELDS:
                assert np.array_equal(got[k], ref[k]), (sched, rep, k)
        g.close()
    plan.close()


def _sparse_set(seed=3):
    """a 16^3 lattice with 45 % of the particles removed and one empty 4^3 block"""
    rng = np.random.default_rng(seed)
    f = inputs.lattice_set(16, seed=seed, jitter=0.1, velocity="gresho", switches=True)
    keep = rng.uniform(size=f["x"].shape[0]) > 0.45
    keep &= ~np.all((f["x"] >= 0.5) & (f["x"] < 0.75), axis=1)
    f = {k: v[keep] for k, v in f.items()}
    # the lattice's h keeps every support inside the adjacent cells of a 4^3 grid
    f, cells, tasks = inputs.uniform_grid(f, 4)
    return inputs.ParticleSet(f, cells, tasks, {"config": -1, "n_side": 16, "grid": 4})


@pytest.mark.parametrize("mode", ["per_task", "batched"])
def test_loops_sparse_and_empty_cells(mode):
    ps = _sparse_set()
    c = ps.cells["count"]
    assert (c == 0).any() and c.max() < 64
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, 8)
    prev = {}
    for loop in range(3):
        if mode == "per_task":
            run_per_task(plan, st, loop, len(ps.tasks), bundle=7)
        else:
            run_batched_loop(plan, st, loop)
        g = outputs(st, loop)
        ref = oracle_loop(ps.fields, loop, prev, epsx=oracle.pack_resolution(ps.cells))
        errs = compare_loop(loop, g, ref)
        log(f"sparse {mode} loop {loop}: {max(errs.values()):.2e}")
        assert max(errs.values()) <= 1e-5, errs
        for k in LOOP_OUT[loop]:
            prev[k] = g[k].astype(np.float64)
    plan.close()


def test_empty_ranges_and_zero_particles():
    import torch
    ps = inputs.make_config(0, n_side=8, grid=4)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, 0)
    before = st.raw()
    buf = torch.empty(256, dtype=torch.uint8, device="cuda")
    for L in range(3):
        sph.sph_pack(plan, L, st, 3, 3, buf)
        sph.INTERACT[L](plan, buf, 3, 3, buf)
        sph.sph_unpack(plan, L, buf, 3, 3, st)
    torch.cuda.synchronize()
    assert st.raw() == before
    # a plan over no particles at all
    cells = np.zeros(0, inputs.CELL_DTYPE)
    tasks = np.zeros(0, inputs.TASK_DTYPE)
    p0 = sph.Plan(cells, tasks, 0)
    st0 = sph.Store(0, 0)
    ws = torch.zeros(sph.sph_batched_ws_bytes(p0) + 256, dtype=torch.uint8, device="cuda")
    sph.sph_step_batched(p0, st0, ws)
    torch.cuda.synchronize()
    p0.close()
    plan.close()


@pytest.mark.parametrize("layout", ["AOS", "SAOS_SHARED", "SOA"])
def test_offload_step_matches_resident_step(layout):
    """host store -> per-loop H2D of the needed substructs -> device step ->
    D2H of the output substructs reproduces the resident batched step bit for
    bit, and leaves every other field of the host store untouched"""
    import torch
    ps = inputs.make_config(1, n_side=32)
    lay = sph.LAYOUTS.index(layout)
    f = dict(ps.fields)
    extra = inputs.random_fields(ps.n, 21, x=f["x"])
    for k in ("time_bin", "id", "cold", "a", "u_dt", "lap_u", "v_sig", "wcount"):
        f[k] = extra[k]
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    resident = sph.Store(lay, ps.n)
    resident.put_all(f)
    sph.sph_step_batched(plan, resident, ws)
    # host store: fill through a device store, then copy the bytes into pinned memory
    host = sph.Store(lay, ps.n, device="pinned")
    tmp = sph.Store(lay, ps.n)
    tmp.put_all(f)
    torch.cuda.synchronize()
    for h, d in zip(host.subs, tmp.subs):
        h.copy_(d.cpu())
    dev = sph.Store(lay, ps.n)
    sph.sph_offload_step(plan, host, dev, ws)
    torch.cuda.synchronize()
    back = sph.Store(lay, ps.n)
    for h, d in zip(host.subs, back.subs):
        d.copy_(h.to("cuda"))
    torch.cuda.synchronize()
    assert back.raw() == resident.raw()
    plan.close()


def _filled_host_store(lay, f, n):
    """a pinned host store holding the fields f (written through a device store)"""
    import torch
    host = sph.Store(lay, n, device="pinned")
    tmp = sph.Store(lay, n)
    tmp.put_all(f)
    torch.cuda.synchronize()
    for h, d in zip(host.subs, tmp.subs):
        h.copy_(d.cpu())
    return host


@pytest.mark.parametrize("layout", ["AOS", "SAOS_SHARED", "SOA"])
def test_offload_async_matches_offload_step(layout):
    """the pipelined offload step (bundles of cells, two copy streams, each
    substruct sent once per step) leaves the host and device stores byte for
    byte as the stream-ordered offload step does, for 1, 3 and 8 bundles, also
    when run twice in a row on one plan"""
    import torch
    ps = inputs.make_config(1, n_side=32)
    lay = sph.LAYOUTS.index(layout)
    f = dict(ps.fields)
    extra = inputs.random_fields(ps.n, 23, x=f["x"])
    for k in ("time_bin", "id", "cold", "a", "u_dt", "lap_u", "v_sig", "wcount"):
        f[k] = extra[k]
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    host_ref = _filled_host_store(lay, f, ps.n)
    dev_ref = sph.Store(lay, ps.n)
    sph.sph_offload_step(plan, host_ref, dev_ref, ws)
    torch.cuda.synchronize()
    ref_h, ref_d = host_ref.raw(), dev_ref.raw()
    for nb in (1, 3, 8):
        log(f"offload async {layout} bundles={nb}")
        host = _filled_host_store(lay, f, ps.n)
        dev = sph.Store(lay, ps.n)
        sph.sph_offload_step_async(plan, host, dev, ws, nbundle=nb)
        torch.cuda.synchronize()
        assert host.raw() == ref_h, nb
        assert dev.raw() == ref_d, nb
    # a second step on the stores the first left behind, both ways
    sph.sph_offload_step(plan, host_ref, dev_ref, ws)
    sph.sph_offload_step_async(plan, host, dev, ws, nbundle=8)
    torch.cuda.synchronize()
    assert host.raw() == host_ref.raw()
    # bundle packs and unpacks split by a loop-fission schedule
    for sched in (2, 4):
        log(f"offload async {layout} bundles=3 schedule={sched}")
        tn = sph.default_tuning()
        tn.pack_schedule = sched
        host_s = _filled_host_store(lay, f, ps.n)
        dev_s = sph.Store(lay, ps.n)
        sph.sph_offload_step_async(plan, host_s, dev_s, ws, nbundle=3, tuning=tn)
        torch.cuda.synchronize()
        assert host_s.raw() == ref_h, sched
        assert dev_s.raw() == ref_d, sched
    plan.close()


def test_layout_choice_and_conversion():
    """the tuner's measured layout choice is the fastest of its own timings,
    and a store converted into it holds the same fields"""
    import torch

    from paper_2606_23891_amd import tune
    ps = inputs.make_config(1, n_side=32)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    log("layout choice")
    best, times = tune.choose_layout(plan, ps.fields, ["AOS", "SAOS_SHARED", "SOA"], log=log)
    assert set(times) == {"AOS", "SAOS_SHARED", "SOA"} and all(t > 0 for t in times.values())
    assert times[best] == min(times.values())
    src = sph.Store(sph.LAYOUTS.index("AOS"), ps.n)
    src.put_all(ps.fields)
    dst = sph.Store(sph.LAYOUTS.index(best), ps.n)
    sph.sph_store_convert(src, dst)
    torch.cuda.synchronize()
    for k in ps.fields:
        assert dst.get(k).tobytes() == src.get(k).tobytes(), k
    plan.close()


def _host_oracle_view(host: "sph.Store", lay: int, n: int):
    """the bytes of a pinned host store read back through the oracle's own
    layout tables"""
    hv = oracle.HostStore(lay, n)
    for dst, src, b in zip(hv.subs, host.subs, hv.sub_bytes):
        dst[:] = src[: n * b].numpy()
    return hv


@pytest.mark.parametrize("layout", ["AOS", "SAOS_SHARED", "SOA"])
def test_offload_forms_against_oracle(layout):
    """after the offload step and the pipelined offload step, the host store
    (read through the oracle's layout tables) holds the loops' outputs within
    the parity tolerance of the oracle (each loop fed the previous loop's
    outputs as the host store holds them), and every field no loop writes
    exactly as it was"""
    import torch

    from gpuhelp import compare_loop, oracle_loop
    ps = inputs.make_config(1, n_side=32)
    lay = sph.LAYOUTS.index(layout)
    f = dict(ps.fields)
    extra = inputs.random_fields(ps.n, 25, x=f["x"])
    for k in ("time_bin", "id", "cold", "a", "u_dt", "lap_u", "v_sig", "wcount"):
        f[k] = extra[k]
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    eps = oracle.pack_resolution(ps.cells)
    written = {"rho", "rho_dh", "wcount", "div_v", "rot_v", "lap_u", "v_sig", "a", "u_dt"}
    for form in ("offload", "offload_async"):
        log(f"{form} {layout} against the oracle")
        host = _filled_host_store(lay, f, ps.n)
        dev = sph.Store(lay, ps.n)
        if form == "offload":
            sph.sph_offload_step(plan, host, dev, ws)
        else:
            sph.sph_offload_step_async(plan, host, dev, ws, nbundle=3)
        torch.cuda.synchronize()
        hv = _host_oracle_view(host, lay, ps.n)
        prev = {}
        for loop in range(3):
            got = {k: hv.get(k) for k in LOOP_OUT[loop]}
            ref = oracle_loop(ps.fields, loop, prev, epsx=eps, grid=True)
            errs = compare_loop(loop, got, ref)
            log(f"{form} loop {loop}: worst {max(errs.values()):.2e}")
            assert max(errs.values()) <= 1e-5, (form, loop, errs)
            for k in LOOP_OUT[loop]:
                prev[k] = got[k].astype(np.float64)
        for k in sph.FIELDS:
            if k not in written:
                assert hv.get(k).tobytes() == np.ascontiguousarray(f[k]).astype(hv.get(k).dtype).tobytes(), (form, k)
    plan.close()


@pytest.mark.parametrize("layout", range(10))
def test_staged_step_matches_per_loop_unpack(layout):
    """the staged step (earlier loops' outputs read from the step's result
    planes, one write-back at the end) leaves the store byte for byte as the
    per-loop pack -> interact -> unpack sequence, both as one call and as its
    seven stage calls; on a 32^3 Gresho lattice with random values in the
    fields no loop touches (padding included)"""
    import torch
    ps = inputs.make_config(1, n_side=32)
    f = dict(ps.fields)
    extra = inputs.random_fields(ps.n, 27, x=f["x"])
    for k in ("time_bin", "id", "cold", "a", "u_dt", "lap_u", "v_sig", "wcount"):
        f[k] = extra[k]
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ref = sph.Store(layout, ps.n)
    for t in ref.subs:
        t.fill_(0x3C)
    ref.put_all(f)
    for L in range(3):
        run_batched_loop(plan, ref, L)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    one = sph.Store(layout, ps.n)
    staged = sph.Store(layout, ps.n)
    for st in (one, staged):
        for t in st.subs:
            t.fill_(0x3C)
        st.put_all(f)
    log(f"staged step {sph.LAYOUTS[layout]}")
    sph.sph_step_batched(plan, one, ws)
    for L in range(3):
        sph.sph_step_pack(plan, L, staged, ws)
        sph.sph_step_interact(plan, L, ws)
    sph.sph_step_writeback(plan, staged, ws)
    torch.cuda.synchronize()
    assert one.raw() == ref.raw()
    assert staged.raw() == ref.raw()
    plan.close()


def _few(xs, vs, h=0.05):
    """a handful of particles in the unit box on a 4^3 grid (most cells empty)"""
    n = len(xs)
    f = {"x": np.array(xs, np.float64), "v": np.array(vs, np.float32), "mass": np.full(n, 1e-3, np.float32),
         "h": np.full(n, h, np.float32), "u": np.linspace(1.0, 2.0, n).astype(np.float32),
         "alpha_v": np.full(n, 0.5, np.float32), "alpha_d": np.full(n, 0.1, np.float32)}
    f, cells, tasks = inputs.uniform_grid(f, 4)
    return inputs.ParticleSet(f, cells, tasks, {"config": -1, "n_side": 0, "grid": 4})


@pytest.mark.parametrize("case", ["single", "pair_one_cell", "pair_across_boundary"])
@pytest.mark.parametrize("mode", ["per_task", "batched", "step"])
def test_single_particle_and_pairs(case, mode):
    """the smallest sets: one particle (density its self term, every gradient
    and force output exactly zero), and two approaching particles, in one cell
    or on either side of the periodic boundary (each loop within 1e-5 of the
    oracle, and the pair's momentum change m_1 a_1 + m_2 a_2 zero to rounding)"""
    import torch
    sets = {"single": ([[0.4, 0.6, 0.3]], [[0.1, -0.2, 0.3]]),
            "pair_one_cell": ([[0.40, 0.60, 0.30], [0.43, 0.62, 0.31]], [[0.5, 0.0, 0.0], [-0.5, 0.1, 0.0]]),
            "pair_across_boundary": ([[0.01, 0.50, 0.50], [0.98, 0.51, 0.49]], [[-0.3, 0.0, 0.0], [0.3, 0.0, 0.1]])}
    ps = _few(*sets[case])
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, sph.LAYOUTS.index("SAOS_SHARED"))
    if mode == "step":
        ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
        sph.sph_step_batched(plan, st, ws)
        torch.cuda.synchronize()
    eps = oracle.pack_resolution(ps.cells)
    prev = {}
    for loop in range(3):
        if mode == "per_task":
            run_per_task(plan, st, loop, len(ps.tasks), bundle=5)
        elif mode == "batched":
            run_batched_loop(plan, st, loop)
        g = outputs(st, loop)
        ref = oracle_loop(ps.fields, loop, prev, epsx=eps)
        errs = compare_loop(loop, g, ref)
        log(f"{case} {mode} loop {loop}: worst {max(errs.values()):.2e}")
        assert max(errs.values()) <= 1e-5, errs
        for k in LOOP_OUT[loop]:
            prev[k] = g[k].astype(np.float64)
    if case == "single":
        assert st.get("rho")[0] > 0 and st.get("wcount")[0] > 0
        for k in ("div_v", "rot_v", "lap_u", "a", "u_dt"):
            assert not np.any(st.get(k)), k
    else:
        assert np.all(st.get("rho") > 0)
        pa = st.get("mass")[:, None].astype(np.float64) * st.get("a").astype(np.float64)
        assert np.abs(pa).max() > 0
        assert np.abs(pa.sum(0)).max() <= 1e-6 * np.abs(pa).max()
    plan.close()
