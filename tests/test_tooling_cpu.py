"""Host-side tooling without a GPU: the rocprofv3 counter summaries that bench
reports traffic from, and the tuning cache keys."""
import csv
import json
import os
import types

import pytest

from paper_2606_23891_amd import profiling, tune

COPY = 'void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(...)>(...)'
FORCE = "void sph::k_interact<2, 1, 128, false>(sph::InteractArgs)"
PREP = "void sph::k_prep<2>(sph::PrepArgs)"


def _write_run(d, counter, values):
    os.makedirs(d, exist_ok=True)
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for i, (k, v) in enumerate(values):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_calibration_and_reload(tmp_path):
    gib = 1 << 30
    # the copy reads 1 GiB but the fetch counter shows half of it; the write counter is exact
    _write_run(tmp_path / "f", "FETCH_SIZE", [(COPY, gib / 2048), (FORCE, 1000.0), (FORCE, 3000.0), (PREP, 512.0)])
    _write_run(tmp_path / "w", "WRITE_SIZE", [(COPY, gib / 1024), (FORCE, 100.0), (FORCE, 100.0), (PREP, 256.0)])
    t = profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), gib)
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    k = t["kernels"][FORCE]
    assert k["dispatches"] == 2
    assert k["fetch_bytes"] == pytest.approx(2000.0 * 1024 * 2)   # mean KiB x 1024 x factor
    assert k["write_bytes"] == pytest.approx(100.0 * 1024)
    assert COPY not in t["kernels"]                                 # only the library's kernels
    md = profiling.traffic_markdown(t, "wl", "cmd f", "cmd w", {FORCE: 1e6})
    p = tmp_path / "summary.md"
    p.write_text(md)
    back = profiling.load_traffic(str(p), "wl")
    assert back is not None and back["kernels"][FORCE]["bytes"] == pytest.approx(k["bytes"])
    assert profiling.load_traffic(str(p), "another workload") is None
    # a summary taken from other kernel sources is not reported
    p.write_text(md.replace(profiling.source_hash(), "0" * 16))
    assert profiling.load_traffic(str(p), "wl") is None


def test_traffic_needs_exactly_one_calibration_copy(tmp_path):
    _write_run(tmp_path / "f", "FETCH_SIZE", [(FORCE, 1.0)])
    _write_run(tmp_path / "w", "WRITE_SIZE", [(FORCE, 1.0)])
    with pytest.raises(RuntimeError):
        profiling.traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 30)


def test_tuning_cache_keys_and_apply(tmp_path, monkeypatch):
    props = types.SimpleNamespace(gcnArchName="gfx950:sramecc+:xnack-", name="", multi_processor_count=256)
    assert tune.device_key(props) == "gfx950-256cu"
    ps = types.SimpleNamespace(meta={"config": 2}, n=16, cells=[0, 1], tasks=[0, 1, 2])
    sig = tune.signature(ps, "SOA")
    assert sig == "cfg2-n16-cells2-tasks3-SOA"
    cache = tmp_path / "cache.json"
    cache.write_text(json.dumps({"gfx950-256cu": {sig: {"window": [512, 256, 128], "blocks_per_cu": 2,
                                                         "blocks_per_loop": [8, 4, 2],
                                                         "queue": 2, "pack_waves": 8,
                                                         "pack_schedule": 3}}}))
    monkeypatch.setattr(tune, "CACHE", str(cache))
    entry = tune.load("gfx950-256cu", sig)
    assert tune.load("gfx942-304cu", sig) is None

    class T:
        window = [0, 0, 0]
        blocks_per_loop = [0, 0, 0]
        blocks_per_cu = pack_waves = queue = pack_schedule = 0
    t = tune.apply(T(), entry)
    assert t.pack_schedule == 3
    assert list(t.window) == [512, 256, 128] and (t.blocks_per_cu, t.queue, t.pack_waves) == (2, 2, 8)
    assert list(t.blocks_per_loop) == [8, 4, 2]


def test_bench_stage_kernel_names():
    """the kernels the benchmark attributes to each stage of the staged step
    (its roofline and traffic lookups use these names)"""
    import importlib.util
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    sys.modules["bench_mod"] = bench
    spec.loader.exec_module(bench)
    t = types.SimpleNamespace(window=[256, 128, 128], pack_schedule=0)
    assert bench.STAGES == ["pack_density", "density", "pack_gradient", "gradient", "pack_force", "force",
                            "writeback"]
    assert bench.stage_kernels("pack_force", 4, t) == ["void sph::k_pack<4, 2, true>(sph::PackArgs)"]
    assert bench.stage_kernels("writeback", 4, t) == ["void sph::k_writeback<4>(sph::UnpackArgs)"]
    assert bench.stage_kernels("force", 4, t) == ["void sph::k_interact<2, 1, 128, false>(sph::InteractArgs)"]
    assert bench.stage_kernels("force", 4, t, mixed=True) == [
        "void sph::k_interact_mixed<1, 128, false>(sph::InteractArgs)"]
    assert bench.stage_kernels("density", 8, t) == ["void sph::k_interact<0, 1, 256, false>(sph::InteractArgs)"]
    # algorithmic bytes per particle: the staged packs read earlier outputs
    # from the result planes and write the derived planes
    shared = [1, 2, 3, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3]   # SAOS_SHARED: packs store rho, rho_dh, D, R
    assert bench.stage_bytes("pack_gradient", 1, shared) == 48 + 4 + 40 + 0.5 + 16 + 4
    assert bench.stage_bytes("pack_force", 1, shared) == 56 + 24 + 68 + 0.5 + 32 + 20
    assert bench.stage_bytes("force", 1, shared) == 68 + 32 + 0.5 + 16
    assert bench.stage_bytes("writeback", 1, shared) == 8 * 7
    assert bench.stage_bytes("writeback", 1, [3] * 13) == 104


def test_fission_table(tmp_path):
    row = lambda tot, rel, pk: {"density": {"pack_ms": 0.1, "unpack_ms": 0.2}, "gradient": {"pack_ms": 0.3,
                                "unpack_ms": 0.4}, "force": {"pack_ms": 0.5, "unpack_ms": 0.6}, "total_ms": tot,
                                "vs_by_particle": rel, "kernels": {"density": [pk, 1], "gradient": [pk, 2],
                                                                   "force": [pk, 3]}}
    out = {"fission": {"SOA": {"by_particle": row(2.1, 1.0, 1), "by_element": row(4.2, 2.0, 5)}}}
    p = tmp_path / "b.log"
    p.write_text("[bench] log line\n" + json.dumps(out) + "\n")
    txt = profiling.fission_markdown(str(p), "T", "python bench.py --fission SOA")
    assert "| layout | by particle | by element |" in txt
    # totals, ratio to the fused kernels, and pack + unpack kernel launches over the three loops
    assert "| SOA | 2.100 (1.00×; 3+6) | 4.200 (2.00×; 15+6) |" in txt
    assert "| SOA | by element | 0.100 / 0.200 | 0.300 / 0.400 | 0.500 / 0.600 |" in txt
