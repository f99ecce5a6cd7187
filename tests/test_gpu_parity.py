"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Pack and unpack: byte equality.  Interaction loops: scaled error
max |q_gpu - q_ref| / max(|q_ref|, sum |terms|) <= 1e-5 (FP32 GPU vs FP64
oracle), signal velocity relative <= 1e-5, interaction counts equal.
"""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

from gpuhelp import (LOOP_OUT, compare_loop, device_store, log, oracle_loop, outputs, run_batched_loop,
                     run_per_task, slot_particles)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _small_sets():
    # uniform 64-per-cell grid, a 512-per-cell grid (multi-tile cells) and an uneven octree
    return {
        "lattice8": inputs.make_config(0, n_side=8, grid=4),
        "grid512": inputs.make_config(2, n_side=32, grid=4),
        "octree": inputs.make_config(3, n_side=24),
    }


@pytest.fixture(scope="module")
def sets():
    return _small_sets()


@pytest.mark.parametrize("layout", range(10))
def test_store_bytes_match_oracle(layout):
    ps = inputs.make_config(0, n_side=8, grid=4)
    f = inputs.random_fields(ps.n, 7, x=ps.fields["x"])
    log(f"store layout={layout}")
    st = sph.Store(layout, ps.n)
    st.put_all(f)
    host = oracle.HostStore(layout, ps.n, fill=0)
    host.put_all(f)
    assert st.raw() == host.raw()
    for k, v in f.items():
        np.testing.assert_array_equal(st.get(k).reshape(v.shape), v)


def _ranges(ntask):
    return [(0, ntask), (0, 1), (ntask // 2, ntask // 2 + 1), (3, min(ntask, 40)), (ntask - 1, ntask), (5, 5)]


@pytest.mark.parametrize("layout", range(10))
def test_pack_bitexact(sets, layout):
    import torch
    for name, ps in sets.items():
        if name != "octree" and layout not in (0, 8):
            continue
        f = inputs.random_fields(ps.n, 11, x=ps.fields["x"])
        st = sph.Store(layout, ps.n)
        st.put_all(f)
        host = oracle.HostStore(layout, ps.n)
        host.put_all(f)
        plan = sph.Plan(ps.cells, ps.tasks, ps.n)
        for loop in range(3):
            for t0, t1 in _ranges(len(ps.tasks)):
                log(f"pack {name} layout={layout} loop={loop} range=[{t0},{t1})")
                ns, pack, res = sph.alloc_range_buffers(plan, loop, t0, t1)
                pack.zero_()
                sph.sph_pack(plan, loop, st, t0, t1, pack)
                torch.cuda.synchronize()
                ref = oracle.pack(host, loop, ps.cells, ps.tasks, t0, t1)
                got = pack.cpu().numpy()[: ref.size]
                assert np.array_equal(got, ref), (name, layout, loop, t0, t1)
        plan.close()


@pytest.mark.parametrize("layout", range(10))
def test_unpack_bitexact(sets, layout):
    import torch
    rng = np.random.default_rng(3)
    for name, ps in sets.items():
        f = inputs.random_fields(ps.n, 13, x=ps.fields["x"])
        plan = sph.Plan(ps.cells, ps.tasks, ps.n)
        nt = len(ps.tasks)
        for loop in range(3):
            st = sph.Store(layout, ps.n)
            st.put_all(f)
            host = oracle.HostStore(layout, ps.n)
            host.put_all(f)
            sph.sph_zero_outputs(plan, loop, st)
            oracle.zero_outputs(host, loop)
            for t0, t1 in [(0, 1), (1, 7), (7, nt // 3), (nt // 3, nt), (4, 4)]:
                log(f"unpack {name} layout={layout} loop={loop} range=[{t0},{t1})")
                ns, pack, res = sph.alloc_range_buffers(plan, loop, t0, t1)
                P = oracle.round_slots(ns)
                r = rng.uniform(-1, 1, (oracle.RESULT_PLANES[loop], P)).astype(np.float32)
                res[: r.nbytes].copy_(torch.from_numpy(r.view(np.uint8).reshape(-1)))
                sph.sph_unpack(plan, loop, res, t0, t1, st)
                oracle.unpack(host, loop, ps.cells, ps.tasks, t0, t1, r)
            assert st.raw() == host.raw(), (name, layout, loop)
        plan.close()


@pytest.mark.parametrize("layout", range(10))
def test_cells_pack_unpack_bitexact(sets, layout):
    import torch
    rng = np.random.default_rng(5)
    for name, ps in sets.items():
        f = inputs.random_fields(ps.n, 17, x=ps.fields["x"])
        plan = sph.Plan(ps.cells, ps.tasks, ps.n)
        assert plan.info().batched_ok
        for loop in range(3):
            log(f"cells pack/unpack {name} layout={layout} loop={loop}")
            st = sph.Store(layout, ps.n)
            st.put_all(f)
            host = oracle.HostStore(layout, ps.n)
            host.put_all(f)
            pack, res = sph.cell_buffers(plan, loop)
            pack.zero_()
            sph.sph_pack_cells(plan, loop, st, pack)
            torch.cuda.synchronize()
            ref = oracle.pack_cells(host, loop, ps.cells)
            assert np.array_equal(pack.cpu().numpy()[: ref.size], ref)
            # the cell pack is the self-task pack of every cell, in cell order
            P = oracle.round_slots(ps.n)
            r = rng.uniform(-1, 1, (oracle.RESULT_PLANES[loop], P)).astype(np.float32)
            r[:, :5] = [-0.0, 0.0, 1e-40, -1e-40, 3.0]   # signed zeros and subnormals
            res[: r.nbytes].copy_(torch.from_numpy(r.view(np.uint8).reshape(-1)))
            sph.sph_unpack_cells(plan, loop, res, st)
            oracle.unpack_cells(host, loop, r)
            assert st.raw() == host.raw()
        plan.close()


@pytest.mark.parametrize("layout", [0, 1, 4, 7, 8, 9])
def test_fission_schedules_bitexact(sets, layout):
    """every loop-fission schedule of the batched pack and unpack writes the
    same bytes as the fused kernels (pack buffers pre-filled with a pattern,
    so a missed or stray write shows) and as the oracle"""
    import torch
    rng = np.random.default_rng(9)
    for name in ("grid512", "octree"):
        ps = sets[name]
        f = inputs.random_fields(ps.n, 19, x=ps.fields["x"])
        plan = sph.Plan(ps.cells, ps.tasks, ps.n)
        for loop in range(3):
            host = oracle.HostStore(layout, ps.n)
            host.put_all(f)
            ref = oracle.pack_cells(host, loop, ps.cells)
            P = oracle.round_slots(ps.n)
            r = rng.uniform(-1, 1, (oracle.RESULT_PLANES[loop], P)).astype(np.float32)
            r[:, :5] = [-0.0, 0.0, 1e-40, -1e-40, 3.0]
            oracle.unpack_cells(host, loop, r)
            fused = None
            for sched in range(5):
                log(f"fission {name} layout={layout} loop={loop} schedule={sched} "
                    f"passes={sph.sph_fission_passes(layout, loop, sched)}")
                tn = sph.default_tuning()
                tn.pack_schedule = sched
                st = sph.Store(layout, ps.n)
                st.put_all(f)
                pack, res = sph.cell_buffers(plan, loop)
                pack.fill_(0x5A)
                sph.sph_pack_cells(plan, loop, st, pack, tn)
                torch.cuda.synchronize()
                got = pack.cpu().numpy()
                if fused is None:
                    fused = got
                assert np.array_equal(got, fused), sched
                pack.zero_()
                sph.sph_pack_cells(plan, loop, st, pack, tn)
                torch.cuda.synchronize()
                assert np.array_equal(pack.cpu().numpy()[: ref.size], ref), sched
                res[: r.nbytes].copy_(torch.from_numpy(r.view(np.uint8).reshape(-1)))
                sph.sph_unpack_cells(plan, loop, res, st, tn)
                torch.cuda.synchronize()
                assert st.raw() == host.raw(), sched
        plan.close()


def test_fission_step_matches_fused_step():
    """a whole batched step under each schedule leaves the store byte for byte
    as the fused step does; an unknown schedule is refused"""
    import torch
    ps = inputs.make_config(1, n_side=32)
    lay = sph.LAYOUTS.index("SAOS_SHARED")
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    ref = None
    for sched in range(5):
        log(f"fission step schedule={sched}")
        tn = sph.default_tuning()
        tn.pack_schedule = sched
        st = device_store(ps, lay)
        sph.sph_step_batched(plan, st, ws, tuning=tn)
        torch.cuda.synchronize()
        ref = st.raw() if ref is None else ref
        assert st.raw() == ref, sched
    tn.pack_schedule = 5
    with pytest.raises(sph.SphError):
        sph.sph_step_batched(plan, st, ws, tuning=tn)
    plan.close()


def test_store_convert_bitexact():
    """converting a store between any two layouts (the same one included)
    leaves the destination byte for byte as the oracle's store of the same
    fields: every member copied, padding zero whatever was there before"""
    import torch
    n = 1000  # ragged: neither a multiple of the 256-thread block nor of 64
    x = inputs.random_fields(n, 29)["x"]
    f = inputs.random_fields(n, 31, x=x)
    refs = {}
    for ld in range(10):
        host = oracle.HostStore(ld, n, fill=0)
        host.put_all(f)
        refs[ld] = host.raw()
    for ls in range(10):
        src = sph.Store(ls, n)
        for t in src.subs:
            t.fill_(0x5A)
        src.put_all(f)
        for ld in range(10):
            log(f"convert {sph.LAYOUTS[ls]} -> {sph.LAYOUTS[ld]} n={n}")
            dst = sph.Store(ld, n)
            for t in dst.subs:
                t.fill_(0xA5)
            sph.sph_store_convert(src, dst)
            torch.cuda.synchronize()
            assert dst.raw() == refs[ld], (ls, ld)
    # refused: different counts, overlapping stores
    small = sph.Store(0, n - 1)
    with pytest.raises(sph.SphError):
        sph.sph_store_convert(src, small)
    with pytest.raises(sph.SphError):
        sph.sph_store_convert(src, src)


def _check_loops(ps, layout, mode, rows=None, bundle=1, tuning=None):
    """density -> gradient -> force on the GPU; each loop compared with the oracle
    fed the GPU's own previous-loop outputs (loop isolation)."""
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    # cells of several widths select the force kernel that tests mixed
    # supports as two matrix-core products
    assert plan.info().mixed_widths == int(np.unique(ps.cells["width"]).size > 1)
    st = device_store(ps, layout)
    prev = {}
    worst = {}
    t = tuning
    if mode == "batched_xcd":
        t = sph.default_tuning()
        t.queue = 2

    def run(loop, counts):
        if mode == "per_task":
            return run_per_task(plan, st, loop, len(ps.tasks), bundle=bundle, counts=counts)
        return run_batched_loop(plan, st, loop, tuning=t, counts=counts)

    for loop in range(3):
        log(f"loops {mode} layout={layout} loop={loop} n={ps.n}")
        # the counting kernels (exact tests, pair counts), then the kernels
        # that run without counts (the ones the benchmark times); both are
        # held to the oracle, and the second feeds the next loop
        cnt = run(loop, True)
        gcnt = outputs(st, loop)
        run(loop, False)
        g = outputs(st, loop)
        ref = oracle_loop(ps.fields, loop, prev, rows=rows, epsx=oracle.pack_resolution(ps.cells), grid=True)
        errs = compare_loop(loop, g, ref, rows=rows)
        for k, e in compare_loop(loop, gcnt, ref, rows=rows).items():
            errs[k] = max(errs[k], e)
        plain = compare_loop(loop, g, ref, rows=rows, plain=True)
        log(f"loop {loop}: plain scaled error, worst {max(plain.values()):.2e}")
        worst.update(errs)
        gc = cnt if rows is None else cnt[rows]
        # counts agree except for pairs within 1e-6 H of the support edge
        dc = np.abs(gc.astype(np.int64) - ref["count"])
        assert np.all(dc <= ref["band"]), (loop, dc.max(), int((dc > ref["band"]).sum()))
        for k in LOOP_OUT[loop]:
            prev[k] = g[k].astype(np.float64)
    plan.close()
    log(f"worst scaled errors: {worst}")
    for k, e in worst.items():
        assert e <= TOL, (k, e, worst)
    return worst


@pytest.mark.parametrize("mode", ["per_task", "batched"])
def test_loops_lattice(mode):
    ps = inputs.make_config(4, n_side=16)
    _check_loops(ps, 8, mode)


@pytest.mark.parametrize("mode", ["per_task", "batched"])
@pytest.mark.parametrize("n_side", [32, 64])
def test_loops_multitile_cells(mode, n_side):
    """4^3 cells of 512 (8 tiles each, 216 j-tiles per cell) and of 4 096
    particles (64 tiles each, 1 728 j-tiles per cell: 27 cull rounds per item)"""
    ps = inputs.make_config(2, n_side=n_side, grid=4)
    rows = np.random.default_rng(1).choice(ps.n, 2048, replace=False)
    _check_loops(ps, 0, mode, rows=rows, bundle=64)


@pytest.mark.parametrize("mode", ["per_task", "batched", "batched_xcd"])
def test_loops_octree_uneven(mode):
    """the clustered set's octree at 64^3: cells of six widths holding 10 to
    2000 particles, supports wider than the smaller cells, tasks between cells
    that are not adjacent; the force loop runs its mixed-support kernel"""
    ps = inputs.make_config(3, n_side=64)
    assert np.unique(ps.cells["width"]).size > 1
    rows = np.random.default_rng(4).choice(ps.n, 8192, replace=False)
    _check_loops(ps, 4, mode, rows=rows, bundle=64)


def _clustered_uniform_grid(n_side=32):
    """the clustered set (supports spanning 90x) on a uniform grid whose cells
    are as wide as the largest support"""
    ps = inputs.make_config(3, n_side=n_side)
    hs = inputs.SUPPORT_PER_H * float(ps.fields["h"].max())
    nc = 4
    while 1.0 / (2 * nc) >= hs:
        nc *= 2
    f, cells, tasks = inputs.uniform_grid(dict(ps.fields), nc)
    return inputs.ParticleSet(f, cells, tasks, {"config": -1, "n_side": n_side, "grid": nc})


@pytest.mark.parametrize("mode", ["per_task", "batched"])
def test_loops_mixed_supports_uniform_grid(mode):
    """mixed supports in the cells of a uniform grid: the force kernel of
    single-width plans then tests each candidate's own support on the VALU"""
    ps = _clustered_uniform_grid()
    assert 1.0 / ps.meta["grid"] >= inputs.SUPPORT_PER_H * float(ps.fields["h"].max())
    h = ps.fields["h"]
    assert h.max() / h.min() > 50
    rows = np.random.default_rng(6).choice(ps.n, 8192, replace=False)
    _check_loops(ps, 4, mode, rows=rows, bundle=64)


def _coincident_set(seed=5):
    """a 16^3 jittered lattice in which 48 particles are moved onto 48 others:
    distinct particles at r = 0, the method's degenerate pair (each keeps its
    own velocity, energy and smoothing length)"""
    rng = np.random.default_rng(seed)
    f = inputs.lattice_set(16, seed=seed, jitter=0.1, velocity="gresho", switches=True)
    src = rng.choice(f["x"].shape[0], 96, replace=False)
    f["x"][src[48:]] = f["x"][src[:48]]
    f, cells, tasks = inputs.uniform_grid(f, 4)
    return inputs.ParticleSet(f, cells, tasks, {"config": -1, "n_side": 16, "grid": 4})


@pytest.mark.parametrize("mode", ["per_task", "batched"])
def test_loops_coincident_particles(mode):
    ps = _coincident_set()
    x = ps.fields["x"]
    assert len(np.unique(x, axis=0)) == x.shape[0] - 48
    _check_loops(ps, 8, mode, bundle=8)


def test_density_closed_form_lattice():
    ps = inputs.make_config(0, jitter=0.0)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, 0)
    run_per_task(plan, st, 0, len(ps.tasks))
    rho = st.get("rho").astype(np.float64)
    np.testing.assert_allclose(rho, 1.0039807860264176, rtol=1e-5)
    run_batched_loop(plan, st, 0)
    np.testing.assert_allclose(st.get("rho").astype(np.float64), 1.0039807860264176, rtol=1e-5)
    plan.close()


def test_batched_work_distribution_bitwise():
    """every tile's sums are formed by one wave in a fixed order, so the
    outputs cannot depend on how tiles are handed out: static stride, one
    queue and per-XCD shares, at two grid sizes, agree bit for bit"""
    import torch

    ps = inputs.make_config(3, n_side=24)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    outs = []
    for queue, bpc in ((0, 1), (1, 4), (2, 2), (2, 16)):
        log(f"work distribution queue={queue} blocks/cu={bpc}")
        st = device_store(ps, 4)
        t = sph.default_tuning()
        t.queue, t.blocks_per_cu = queue, bpc
        for loop in range(3):
            run_batched_loop(plan, st, loop, tuning=t)
        torch.cuda.synchronize()
        outs.append(st.raw())
    plan.close()
    for o in outs[1:]:
        assert o == outs[0]


def _chain_ref(ps, eps):
    """the oracle's own FP64 chain: density, then gradient with its own rho,
    then force with its own rho, rho_dh, D and R"""
    f = ps.fields
    d = oracle.density(f["x"], f["mass"], f["h"], epsx=eps, grid=True)
    g = oracle.gradient(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"], epsx=eps, grid=True)
    fo = oracle.force(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"], d["rho_dh"], g["div_v"], g["rot_v"],
                      f["alpha_v"], f["alpha_d"], epsx=eps, grid=True)
    return [d, g, fo]


@pytest.mark.parametrize("k,n_side,loops", [(0, None, 1), (1, 32, 3), (4, 32, 3)])
def test_full_fp64_chain(k, n_side, loops):
    """the whole step on the GPU (batched, one call) against the oracle's own
    FP64 chain, where every loop reads the oracle's previous-loop outputs
    rather than the GPU's: the 16^3 lattice (density only, its workload), the
    32^3 Gresho lattice and the 32^3 adjoint lattice"""
    import torch
    ps = inputs.make_config(k, n_side=n_side) if n_side else inputs.make_config(k)
    eps = oracle.pack_resolution(ps.cells)
    refs = _chain_ref(ps, eps)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, sph.LAYOUTS.index("SAOS_SHARED"))
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    sph.sph_step_batched(plan, st, ws)
    torch.cuda.synchronize()
    for loop in range(loops):
        errs = compare_loop(loop, outputs(st, loop), refs[loop])
        plain = compare_loop(loop, outputs(st, loop), refs[loop], plain=True)
        log(f"chain cfg{k} loop {loop}: worst {max(errs.values()):.2e} {errs}")
        log(f"chain cfg{k} loop {loop}: plain scaled error, worst {max(plain.values()):.2e} {plain}")
        assert max(errs.values()) <= TOL, (loop, errs)
        if loop == 0:
            assert max(plain.values()) <= TOL, plain
    plan.close()


def _bench_entries():
    """every tuning-cache entry of this device (the launch parameters the
    benchmark runs with on its workloads)"""
    import json
    import os

    import torch

    from paper_2606_23891_amd import tune
    data = json.load(open(tune.CACHE)) if os.path.exists(tune.CACHE) else {}
    return data.get(tune.device_key(torch.cuda.get_device_properties(0)), {})


@pytest.mark.parametrize("which", ["lattice", "grid512", "octree"])
def test_loops_benchmark_tunings(which):
    """the kernel variants and launch parameters of every benchmark tuning
    entry (windows, work queues, waves per CU) on the small sets, against the
    oracle"""
    ps = {"lattice": lambda: inputs.make_config(4, n_side=16),
          "grid512": lambda: inputs.make_config(2, n_side=32, grid=4),
          "octree": lambda: inputs.make_config(3, n_side=24)}[which]()
    rows = None if ps.n <= 8192 else np.random.default_rng(2).choice(ps.n, 4096, replace=False)
    entries = _bench_entries()
    assert entries, "no tuning-cache entry for this device"
    from paper_2606_23891_amd import tune
    for sig, entry in entries.items():
        t = tune.apply(sph.default_tuning(), entry)
        log(f"tuning {sig}: {entry}")
        _check_loops(ps, sph.LAYOUTS.index("SAOS_SHARED"), "batched", rows=rows, tuning=t)
