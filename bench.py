"""Benchmark of the SPH pack / interact / unpack hot path on one MI355X.

One step = density -> gradient -> force, each as pack -> interaction, then
one write-back of every output (the unpacks folded into one pass at the end
of the step), over the whole synthetic workload (inputs resident in HBM).
The timed region runs the batched step stage by stage on one stream with HIP
events between the seven stages, so every kernel's average duration is
measured inside the timed region.  Reported beside it: the same step replayed as one
captured HIP graph, the per-task form (one launch per task and stage, the
paper's offload cycle with single-task bundles), and the CPU oracle timed on
a bounded sample of the same workload.

Prints one JSON line.  Default workload: the 256^3 Gresho-vortex set on a 32^3
cell grid (16 777 216 particles, 458 752 tasks).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + pack/unpack GB/s (batched vs per-task, FP32 @1e-5 rel)"
# FP32 operations the pair body of each loop executes per interacting pair
# (add, mul, min/max, sqrt, rsqrt, rcp = 1; fma = 2; the candidate test excluded)
PAIR_FLOPS = {0: 32, 1: 55, 2: 81}
# the same per-pair work as fixed beforehand from the SPH formulas (a textbook
# count of the terms, independent of this implementation's folding)
PAIR_FLOPS_FORMULA = {0: 18, 1: 50, 2: 110}
# algorithmic HBM bytes per particle, per-loop form: fields read from the
# store + packed record written (+ 32 bytes of tile bounds per 64 particles);
# unpack: result read + outputs written
PACK_BYTES = {0: 32 + 20 + 0.5, 1: 52 + 40 + 0.5, 2: 80 + 68 + 0.5}
UNPACK_BYTES = {0: 12 + 12, 1: 24 + 24, 2: 16 + 16}
# staged step: the gradient / force packs read the fields earlier loops of the
# step produce from its result planes (4 / 24 bytes) instead of the store, and
# write the derived planes of the pair term (16 / 32 bytes); each of the 13
# outputs is stored once, 4 bytes, by the stage the library names for the
# store's layout (a pack that loads the output's record whole, else the
# write-back, which also reads the output's result, 4 bytes)
STEP_PACK_BYTES = {0: 32 + 20 + 0.5, 1: 48 + 4 + 40 + 0.5 + 16, 2: 56 + 24 + 68 + 0.5 + 32}
OUTPUT_BYTES = 4
# interaction kernel: its packed records and derived planes read once + its
# result planes written
INTERACT_BYTES = {0: 20 + 0.5 + 12, 1: 40 + 16 + 0.5 + 24, 2: 68 + 32 + 0.5 + 16}
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
LOOP_NAME = {0: "density", 1: "gradient", 2: "force"}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, help="workload 1..3 (2: 256^3 Gresho)")
    ap.add_argument("--grid", type=int, default=None, help="cells per side (uniform workloads)")
    ap.add_argument("--n-side", type=int, default=None)
    ap.add_argument("--layout", default="SAOS_SHARED")
    ap.add_argument("--per-task", default="auto", help="auto | full | off | <tasks> (sampled, scaled)")
    ap.add_argument("--per-task-budget", type=float, default=40.0, help="seconds for the per-task leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--layouts", default=None,
                    help="'all' or comma list: also time pack + unpack of every loop per store layout")
    ap.add_argument("--fission", default=None,
                    help="'all' or comma list of layouts: also time pack + unpack under every "
                         "loop-fission schedule")
    ap.add_argument("--adjoint", default=None,
                    help="comma list of lattice sides: also time the adjoint (forward, forward + backward) on "
                         "the Gresho lattice of that many particles per side")
    ap.add_argument("--kdk", action="store_true",
                    help="also time kick-drift-kick steps (CFL time step) around the loops")
    ap.add_argument("--hiter", action="store_true",
                    help="also time the smoothing-length iteration from h perturbed by up to 10 %%")
    ap.add_argument("--convert", default=None,
                    help="'default' or comma list of SRC:DST layouts: also time whole-store layout "
                         "conversions")
    ap.add_argument("--offload", default=None,
                    help="'all' or comma list of layouts: also time the offload form (pinned host store)")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the plain elementwise copy timed after the step (the achievable-HBM "
                         "reference, and the calibration dispatch of HBM-traffic counter runs)")
    ap.add_argument("--tuning", default="auto",
                    help="auto (the tuner's cache for this device and workload, else defaults), "
                         "default, or a JSON file with sph_tuning fields")
    return ap.parse_args()


TRAFFIC_SUMMARY = "hbm_traffic_gresho256.md"


def stage_kernels(stage, layout, tuning, mixed=False):
    """the kernels a stage of the staged batched step launches (demangled
    names; the queue reset of the interaction stages, a one-thread kernel, is
    left out); mixed: the plan's cells differ in width, so the force loop runs
    its mixed-support kernel"""
    if stage == "writeback":
        return [f"void sph::k_writeback<{layout}>(sph::UnpackArgs)"]
    for L, nm in LOOP_NAME.items():
        if stage == f"pack_{nm}":
            return [f"void sph::k_pack<{layout}, {L}, true>(sph::PackArgs)"]
        if stage == nm:
            if L == 2 and mixed:
                return [f"void sph::k_interact_mixed<1, {tuning.window[L]}, false>(sph::InteractArgs)"]
            return [f"void sph::k_interact<{L}, 1, {tuning.window[L]}, false>(sph::InteractArgs)"]
    raise KeyError(stage)


def stage_bytes(stage, n, writers):
    """algorithmic HBM bytes of one launch of a stage of the staged step;
    writers: the stage storing each output (1, 2: that loop's pack; 3: the
    write-back), from the library for the store's layout"""
    if stage == "writeback":
        return 2 * OUTPUT_BYTES * sum(1 for w in writers if w == 3) * n
    for L, nm in LOOP_NAME.items():
        if stage == f"pack_{nm}":
            return (STEP_PACK_BYTES[L] + OUTPUT_BYTES * sum(1 for w in writers if w == L)) * n
        if stage == nm:
            return INTERACT_BYTES[L] * n
    raise KeyError(stage)


STAGES = ["pack_density", "density", "pack_gradient", "gradient", "pack_force", "force", "writeback"]


def workload_name(k, ps):
    st = ps.meta
    kind = {1: "gresho", 2: "gresho", 3: "clustered-octree"}.get(k, f"cfg{k}")
    g = st.get("grid")
    cells = f"{g}^3 cells" if g else f"{len(ps.cells)} octree leaves"
    return f"{kind}-{st['n_side']}^3 ({ps.n} particles), {cells}, {len(ps.tasks)} tasks"


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the library has no "
                                   "multi-GPU path (how it would shard is described in the design notes)",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2606_23891_amd import inputs, sph

    torch.cuda.set_device(0)
    dev = torch.cuda.get_device_properties(0)
    t0 = time.time()
    kw = {}
    if a.grid:
        kw["grid"] = a.grid
    if a.n_side:
        kw["n_side"] = a.n_side
    ps = inputs.make_config(a.config, **kw)
    log(f"workload built in {time.time() - t0:.1f}s: n={ps.n} cells={len(ps.cells)} tasks={len(ps.tasks)}")
    layout = sph.LAYOUTS.index(a.layout)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    info = plan.info()
    store = sph.Store(layout, ps.n)
    store.put_all(ps.fields)
    from paper_2606_23891_amd import tune

    tuning = sph.default_tuning()
    tuned_from = "defaults"
    if a.tuning == "auto":
        entry = tune.load(tune.device_key(dev), tune.signature(ps, a.layout))
        if entry:
            tune.apply(tuning, entry)
            tuned_from = "tuning cache"
    elif a.tuning != "default":
        tune.apply(tuning, json.load(open(a.tuning)))
        tuned_from = a.tuning
    if tuning.pack_schedule != 0:
        log("the staged step packs each loop in one kernel: the tuning's loop-fission schedule is not used")
        tuning.pack_schedule = 0
    log(f"tuning ({tuned_from}): blocks/CU {tuning.blocks_per_cu} per loop {list(tuning.blocks_per_loop)} "
        f"windows {list(tuning.window)} queue {tuning.queue} pack waves {tuning.pack_waves}")
    params = sph.default_params()
    stream = torch.cuda.current_stream()
    bufs = {L: sph.cell_buffers(plan, L) for L in range(3)}
    ws = sph.interact_ws(plan)
    sws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")

    def stage(i):
        # the staged step: pack and interactions per loop, one write-back
        if i == 6:
            sph.sph_step_writeback(plan, store, sws, tuning=tuning)
        elif i % 2 == 0:
            sph.sph_step_pack(plan, i // 2, store, sws, params=params, tuning=tuning)
        else:
            sph.sph_step_interact(plan, i // 2, sws, params=params, tuning=tuning)

    # interaction counts (untimed, per-loop form with the counting kernels)
    pairs = {}
    cnt = torch.zeros(ps.n, dtype=torch.int32, device="cuda")
    for L in range(3):
        pack, res = bufs[L]
        sph.sph_pack_cells(plan, L, store, pack, tuning)
        sph.sph_interact_cells(plan, L, pack, res, ws, params=params, tuning=tuning, counts=cnt)
        sph.sph_unpack_cells(plan, L, res, store, tuning)
        torch.cuda.synchronize()
        pairs[L] = int(cnt.to(torch.int64).sum().item())
    total_pairs = sum(pairs.values())
    log(f"interacting pairs per step: {pairs}")
    del bufs, ws
    torch.cuda.empty_cache()

    for _ in range(a.warmup):
        for i in range(7):
            stage(i)
    torch.cuda.synchronize()

    # timed region: K steps, events between all 7 stages
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(8)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for k in range(a.steps):
        ev[k][0].record(stream)
        for i in range(7):
            stage(i)
            ev[k][i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    stage_ms = np.zeros(7)
    step_ms = []
    for k in range(a.steps):
        for i in range(7):
            stage_ms[i] += ev[k][i].elapsed_time(ev[k][i + 1])
        step_ms.append(ev[k][0].elapsed_time(ev[k][7]))
    stage_ms /= a.steps
    ms_per_step = float(np.mean(step_ms))
    value = total_pairs / (ms_per_step * 1e-3)
    log(f"batched: {ms_per_step:.3f} ms/step (wall {1e3 * wall / a.steps:.3f}), {value:.3e} pairs/s")

    stages = {}
    n = ps.n
    writers = sph.sph_step_output_writers(layout)
    for i, nm in enumerate(STAGES):
        ms = float(stage_ms[i])
        if nm in LOOP_NAME.values():
            L = [k for k, v in LOOP_NAME.items() if v == nm][0]
            stages[nm] = {"ms": ms, "pairs": pairs[L],
                          "TFLOP/s": PAIR_FLOPS[L] * pairs[L] / (ms * 1e-3) / 1e12,
                          "TFLOP/s_formula_count": PAIR_FLOPS_FORMULA[L] * pairs[L] / (ms * 1e-3) / 1e12,
                          "pairs/s": pairs[L] / (ms * 1e-3),
                          "GB/s": stage_bytes(nm, n, writers) / (ms * 1e-3) / 1e9}
        else:
            stages[nm] = {"ms": ms, "GB/s": stage_bytes(nm, n, writers) / (ms * 1e-3) / 1e9}
    pu = [k for k in STAGES if k.startswith("pack_") or k == "writeback"]
    pu_bytes = sum(stage_bytes(k, n, writers) for k in pu)
    pu_ms = sum(stages[k]["ms"] for k in pu)
    pack_unpack_gbs = pu_bytes / (pu_ms * 1e-3) / 1e9

    # dominant kernel and its roofline
    names = list(stages)
    dom = names[int(np.argmax([stages[k]["ms"] for k in names]))]
    if "TFLOP/s" not in stages[dom]:
        roof = {"kernel": dom, "bound": "hbm", "achieved": stages[dom]["GB/s"], "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": stages[dom]["TFLOP/s"], "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "flops_per_pair": PAIR_FLOPS[names.index(dom) // 2],
                "achieved_formula_count": stages[dom]["TFLOP/s_formula_count"],
                "flops_per_pair_formula_count": PAIR_FLOPS_FORMULA[names.index(dom) // 2],
                "kernel_ms": stages[dom]["ms"]}
        roof["frac_formula_count"] = roof["achieved_formula_count"] / roof["peak"]
    roof["frac"] = roof["achieved"] / roof["peak"]
    # HBM bytes per launch of that kernel from the committed counter summary of
    # this workload, if it was taken from the current kernel sources
    from paper_2606_23891_amd import profiling

    wl = f"{workload_name(a.config, ps)}; {a.layout}"
    tr = profiling.load_traffic(os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY), wl)
    knames = stage_kernels(dom, layout, tuning, mixed=bool(info.mixed_widths))
    roof["kernels"] = knames
    roof["traffic"] = (sum(tr["kernels"][k]["bytes"] for k in knames)
                       if tr and all(k in tr["kernels"] for k in knames) else None)
    roof["traffic_unit"] = "bytes per launch of the stage's kernels"
    roof["algorithmic_bytes"] = stage_bytes(dom, n, writers)

    out = {
        "metric": METRIC, "value": value, "unit": "pair interactions/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_per_step, "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload_name(a.config, ps), "layout": a.layout, "form": "batched, staged",
                   "pairs_per_step": total_pairs, "device": tune.device_key(dev), "cu": dev.multi_processor_count,
                   "tuning": {"source": tuned_from, "blocks_per_cu": tuning.blocks_per_cu,
                              "blocks_per_loop": list(tuning.blocks_per_loop),
                              "window": list(tuning.window), "queue": tuning.queue,
                              "pack_waves": tuning.pack_waves}},
        "pack_unpack_GBps": pack_unpack_gbs,
        "stages": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                   for k, v in stages.items()},
        "roofline": roof,
    }

    # a plain elementwise copy (read + write of copy_mib MiB each) on the same stream
    if a.copy_mib > 0:
        src = torch.zeros(a.copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.neg(src, out=dst)
        e0.record(stream)
        for _ in range(3):
            torch.neg(src, out=dst)
        e1.record(stream)
        torch.cuda.synchronize()
        out["hbm_copy_GBps"] = 2 * (a.copy_mib << 20) * 3 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        log(f"plain copy: {out['hbm_copy_GBps']:.0f} GB/s")
        del src, dst

    # the same step as one captured graph
    if not a.no_graph:
        wsb = sws
        g = sph.Graph(plan, store, wsb, params=params, tuning=tuning)
        g.launch(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(a.steps):
            g.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        out["graph_ms_per_step"] = e0.elapsed_time(e1) / a.steps
        g.close()
        del wsb
        log(f"graph: {out['graph_ms_per_step']:.3f} ms/step")

    # the per-task form
    if a.per_task != "off":
        ntask = len(ps.tasks)
        pb, rb = 0, 0
        for L in range(3):
            p_, r_ = sph.sph_plan_task_max_bytes(plan, L)
            pb, rb = max(pb, p_), max(rb, r_)
        pbuf = torch.empty(pb, dtype=torch.uint8, device="cuda")
        rbuf = torch.empty(rb, dtype=torch.uint8, device="cuda")
        # probe the launch rate on a slice, then run all tasks or a scaled sample
        probe = min(ntask, 2048)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        sph.sph_run_per_task(plan, 0, store, 0, probe, pbuf, rbuf, params=params)
        torch.cuda.synchronize()
        e0.record(stream)
        for L in range(3):
            sph.sph_run_per_task(plan, L, store, 0, probe, pbuf, rbuf, params=params)
        e1.record(stream)
        torch.cuda.synchronize()
        est = e0.elapsed_time(e1) / probe * ntask / 1e3
        if a.per_task == "full" or (a.per_task == "auto" and est <= a.per_task_budget):
            nt = ntask
        elif a.per_task == "auto":
            nt = max(probe, int(ntask * a.per_task_budget / est))
        else:
            nt = min(ntask, int(a.per_task))
        e0.record(stream)
        for L in range(3):
            sph.sph_run_per_task(plan, L, store, 0, nt, pbuf, rbuf, params=params)
        e1.record(stream)
        torch.cuda.synchronize()
        pt_ms = e0.elapsed_time(e1) * ntask / nt
        out["per_task_ms_per_step"] = pt_ms
        out["per_task_tasks_timed"] = nt
        out["per_task_scaled"] = nt < ntask
        out["batched_speedup_vs_per_task"] = pt_ms / ms_per_step
        log(f"per-task: {pt_ms:.1f} ms/step ({nt}/{ntask} tasks timed)")
        del pbuf, rbuf

    # pack + unpack per store layout (the paper's layout comparison, on HBM)
    if a.layouts:
        names = sph.LAYOUTS if a.layouts == "all" else a.layouts.split(",")
        out["layouts"] = layout_sweep(ps, plan, names, tuning, a.steps)

    if a.fission:
        names = sph.LAYOUTS if a.fission == "all" else a.fission.split(",")
        out["fission"] = fission_sweep(ps, plan, names, tuning, a.steps)

    if a.adjoint:
        out["adjoint"] = [adjoint_bench(int(k)) for k in a.adjoint.split(",")]

    if a.kdk:
        out["kdk"] = kdk_bench(ps, plan, tuning, a.layout, a.steps)

    if a.hiter:
        out["h_iteration"] = hiter_bench(ps, plan, tuning, a.layout)

    if a.convert:
        pairs = CONVERT_PAIRS if a.convert == "default" else [tuple(x.split(":")) for x in a.convert.split(",")]
        out["convert"] = convert_sweep(ps, pairs, a.steps)

    if a.offload:
        names = sph.LAYOUTS if a.offload == "all" else a.offload.split(",")
        out["offload"] = offload_sweep(ps, plan, names, tuning)

    # the CPU oracle on a bounded sample of the same workload
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(ps, store, a.cpu_seconds, a.layout)

    print(json.dumps(out), flush=True)


def _pack_unpack_row(ps, plan, st, bufs, tuning, steps):
    """pack + unpack time of each loop of the batched form on one store"""
    import torch

    from paper_2606_23891_amd import sph

    stream = torch.cuda.current_stream()
    row = {}
    for L in range(3):
        pack, r = bufs[L]
        for s_ in range(2):
            sph.sph_pack_cells(plan, L, st, pack, tuning)
            sph.sph_unpack_cells(plan, L, r, st, tuning)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        tp = tu = 0.0
        for _ in range(steps):
            e[0].record(stream)
            sph.sph_pack_cells(plan, L, st, pack, tuning)
            e[1].record(stream)
            sph.sph_unpack_cells(plan, L, r, st, tuning)
            e[2].record(stream)
            torch.cuda.synchronize()
            tp += e[0].elapsed_time(e[1])
            tu += e[1].elapsed_time(e[2])
        tp /= steps
        tu /= steps
        row[LOOP_NAME[L]] = {"pack_ms": round(tp, 4), "unpack_ms": round(tu, 4),
                             "pack_GB/s": round(PACK_BYTES[L] * ps.n / (tp * 1e-3) / 1e9, 1),
                             "unpack_GB/s": round(UNPACK_BYTES[L] * ps.n / (tu * 1e-3) / 1e9, 1)}
    row["total_ms"] = round(sum(v["pack_ms"] + v["unpack_ms"] for k, v in row.items() if k in LOOP_NAME.values()), 4)
    return row


def _staged_row(ps, plan, st, sws, tuning, steps):
    """the staged step's conversions on one store: the three packs (earlier
    outputs from the step's result planes, derived planes written) and the
    write-back, the interactions left out (the result planes keep whatever a
    previous step left there: the timing does not depend on their values)"""
    import torch

    from paper_2606_23891_amd import sph

    stream = torch.cuda.current_stream()
    writers = sph.sph_step_output_writers(st.layout)
    stages = ["pack_density", "pack_gradient", "pack_force", "writeback"]

    def run(i):
        if i == 3:
            sph.sph_step_writeback(plan, st, sws, tuning=tuning)
        else:
            sph.sph_step_pack(plan, i, st, sws, tuning=tuning)

    for i in range(4):
        run(i)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    acc = np.zeros(4)
    for _ in range(steps):
        ev[0].record(stream)
        for i in range(4):
            run(i)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        acc += [ev[i].elapsed_time(ev[i + 1]) for i in range(4)]
    acc /= steps
    row = {nm: {"ms": round(float(ms), 4), "GB/s": round(stage_bytes(nm, ps.n, writers) / (ms * 1e-3) / 1e9, 1)}
           for nm, ms in zip(stages, acc)}
    row["total_ms"] = round(float(acc.sum()), 4)
    return row


def layout_sweep(ps, plan, names, tuning, steps):
    """pack + unpack time of each loop for every store layout (fresh store
    each), per-loop form, and the staged step's packs + write-back"""
    import torch

    from paper_2606_23891_amd import sph

    bufs = {L: sph.cell_buffers(plan, L) for L in range(3)}
    sws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    res = {}
    for name in names:
        st = sph.Store(sph.LAYOUTS.index(name), ps.n)
        st.put_all(ps.fields)
        torch.cuda.synchronize()
        row = _pack_unpack_row(ps, plan, st, bufs, tuning, steps)
        row["staged"] = _staged_row(ps, plan, st, sws, tuning, steps)
        res[name] = row
        log(f"layout {name}: pack+unpack {row['total_ms']:.3f} ms per step")
        del st
        torch.cuda.empty_cache()
    base = res.get("AOS", {}).get("total_ms")
    if base:
        for name in res:
            res[name]["vs_AOS"] = round(res[name]["total_ms"] / base, 4)
    return res


def fission_sweep(ps, plan, names, tuning, steps):
    """pack + unpack time per loop-fission schedule of the batched form, for
    each named store layout (Sec. 3.3's split conversion loops, one kernel per
    group of members)"""
    import copy

    import torch

    from paper_2606_23891_amd import sph

    bufs = {L: sph.cell_buffers(plan, L) for L in range(3)}
    res = {}
    for name in names:
        lay = sph.LAYOUTS.index(name)
        st = sph.Store(lay, ps.n)
        st.put_all(ps.fields)
        torch.cuda.synchronize()
        res[name] = {}
        for sname, sched in sph.SCHEDULES.items():
            tn = copy.copy(tuning) if tuning is not None else sph.default_tuning()
            tn.pack_schedule = sched
            row = _pack_unpack_row(ps, plan, st, bufs, tn, steps)
            row["kernels"] = {LOOP_NAME[L]: [len(m) for m in sph.sph_fission_passes(lay, L, sched)]
                              for L in range(3)}
            res[name][sname] = row
            log(f"fission {name} {sname}: pack+unpack {row['total_ms']:.3f} ms per step")
        base = res[name]["by_particle"]["total_ms"]
        for sname in res[name]:
            res[name][sname]["vs_by_particle"] = round(res[name][sname]["total_ms"] / base, 4)
        del st
        torch.cuda.empty_cache()
    return res


def adjoint_bench(n_side, reps=5):
    """forward (accelerations in FP64 from float64 positions) and forward +
    backward (hand-written adjoint kernels) of the autograd Function, L =
    sum |a|^2, on the jittered Gresho lattice with a velocity dispersion; the
    viscosity switch is held at the fields' alpha_v (the adjoint treats it as
    a constant, so its value does not change the work)"""
    import numpy as np
    import torch

    from paper_2606_23891_amd import autograd, inputs, sph

    ps = inputs.make_config(4, n_side=n_side)
    f = ps.fields
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    T = lambda arr, dt: torch.tensor(np.ascontiguousarray(arr), dtype=dt, device="cuda")
    ctx = autograd.make_context(plan, T(f["h"], torch.float32), T(f["u"], torch.float32),
                                T(f["alpha_v"], torch.float32), T(f["alpha_d"], torch.float32))
    x = T(f["x"], torch.float64).requires_grad_(True)
    v = T(f["v"], torch.float32).requires_grad_(True)
    m = T(f["mass"], torch.float32).requires_grad_(True)
    stream = torch.cuda.current_stream()

    def fwd():
        with torch.no_grad():
            return autograd.acceleration(x, v, m, ctx)

    def fwd_bwd():
        a = autograd.acceleration(x, v, m, ctx)
        (a.double() ** 2).sum().backward()

    res = {"n": ps.n, "workload": f"gresho-{n_side}^3 lattice, velocity dispersion 0.02"}
    for name, fn in (("forward_ms", fwd), ("forward_backward_ms", fwd_bwd)):
        for _ in range(3):   # untimed: a process's first backward passes run slower (one-time set-up)
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        res[name] = round(e0.elapsed_time(e1) / reps, 3)
    res["backward_over_forward"] = round((res["forward_backward_ms"] - res["forward_ms"]) / res["forward_ms"], 3)
    log(f"adjoint {n_side}^3: forward {res['forward_ms']:.2f} ms, forward+backward {res['forward_backward_ms']:.2f} ms")
    plan.close()
    del ctx, x, v, m
    torch.cuda.empty_cache()
    return res


def kdk_bench(ps, plan, tuning, layout_name, steps, cfl=0.1):
    """kick-drift-kick steps on a fresh store: dt from the CFL condition of the
    first state, then `steps` timed steps (each synchronises once)"""
    import time

    import torch

    from paper_2606_23891_amd import sph

    st = sph.Store(sph.LAYOUTS.index(layout_name), ps.n)
    st.put_all(ps.fields)
    ws = torch.empty(sph.kdk_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    sws = ws[: sph.sph_batched_ws_bytes(plan)]
    iws = ws[(sph.sph_batched_ws_bytes(plan) + 255) // 256 * 256:]
    sph.sph_step_batched(plan, st, sws, tuning=tuning)
    dt = sph.sph_cfl_dt(plan, st, iws, cfl=cfl)
    sph.sph_step_kdk(plan, st, ws, dt, tuning=tuning)   # warm-up step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sph.sph_step_kdk(plan, st, ws, dt, tuning=tuning)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    mo, mh = sph.sph_drift(plan, st, 0.0, iws)
    res = {"ms_per_step": round(ms, 3), "dt": dt, "cfl": cfl, "steps": steps,
           "max_outside_cell": mo, "max_h": mh}
    log(f"kdk: {ms:.3f} ms per step (dt {dt:.3e}, {steps} steps)")
    del st, ws
    torch.cuda.empty_cache()
    return res


def hiter_bench(ps, plan, tuning, layout_name, eta=1.2348, tol=1e-4):
    """the smoothing-length iteration on the workload, every h first scaled by a
    seeded factor in [0.9, 1.1]: passes, particles left moving, wall time"""
    import time

    import numpy as np
    import torch

    from paper_2606_23891_amd import sph

    st = sph.Store(sph.LAYOUTS.index(layout_name), ps.n)
    st.put_all(ps.fields)
    h0 = (ps.fields["h"] * np.random.default_rng(17).uniform(0.9, 1.1, ps.n)).astype(np.float32)
    ws = torch.empty(sph.sph_h_iterate_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    res = {}
    for rep in range(2):   # the first call warms up
        st.put("h", h0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        passes, still = sph.sph_h_iterate(plan, st, ws, eta=eta, tol=tol, max_iter=30, tuning=tuning)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res = {"passes": passes, "unconverged": still, "ms": round(ms, 3), "ms_per_pass": round(ms / passes, 3),
               "eta": eta, "tol": tol, "start": "h x U(0.9, 1.1), seed 17"}
    log(f"h iteration: {res['passes']} passes, {res['unconverged']} unconverged, {res['ms']:.2f} ms")
    del st, ws
    torch.cuda.empty_cache()
    return res


CONVERT_PAIRS = [("AOS", "SOA"), ("SOA", "AOS"), ("AOS", "SAOS_SHARED"), ("SAOS_SHARED", "AOS"),
                 ("SAOS_SHARED", "SOA"), ("SOA", "SAOS_SHARED"), ("SAOS_SHARED", "SAOS_SHARED")]


def convert_sweep(ps, pairs, steps):
    """whole-store layout conversion: time and rate (every record of both
    stores moved once)"""
    import torch

    from paper_2606_23891_amd import sph

    stream = torch.cuda.current_stream()
    res = {}
    stores = {}
    for src_name, dst_name in pairs:
        for nm in (src_name, dst_name):
            if nm not in stores:
                stores[nm] = sph.Store(sph.LAYOUTS.index(nm), ps.n)
                stores[nm].put_all(ps.fields)
        src = stores[src_name]
        dst = stores[dst_name] if dst_name != src_name else sph.Store(sph.LAYOUTS.index(dst_name), ps.n)
        sph.sph_store_convert(src, dst)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            sph.sph_store_convert(src, dst)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        nbytes = ps.n * (sum(sph.sph_layout_info(src.layout)) + sum(sph.sph_layout_info(dst.layout)))
        res[f"{src_name}->{dst_name}"] = {"ms": round(ms, 4), "bytes": nbytes,
                                          "GB/s": round(nbytes / (ms * 1e-3) / 1e9, 1)}
        log(f"convert {src_name} -> {dst_name}: {ms:.3f} ms, {nbytes / (ms * 1e-3) / 1e9:.0f} GB/s")
    del stores
    torch.cuda.empty_cache()
    return res


def offload_sweep(ps, plan, names, tuning, reps=2):
    """the offload form per layout: host store in pinned memory, per-loop copies
    of the substructs each loop needs, batched compute on the device; also the
    pipelined step (4 and 16 bundles of cells, copies on two streams)"""
    import torch

    from paper_2606_23891_amd import sph

    stream = torch.cuda.current_stream()
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    res = {}
    for name in names:
        lay = sph.LAYOUTS.index(name)
        dev = sph.Store(lay, ps.n)
        dev.put_all(ps.fields)
        host = sph.Store(lay, ps.n, device="pinned")
        for h, d in zip(host.subs, dev.subs):
            h.copy_(d.cpu())
        h2d = d2h = 0
        for L in range(3):
            a_, b_ = sph.sph_offload_bytes(lay, L, ps.n)
            h2d += a_
            d2h += b_
        sph.sph_offload_step(plan, host, dev, ws, tuning=tuning)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            sph.sph_offload_step(plan, host, dev, ws, tuning=tuning)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms_per_step": round(ms, 3), "h2d_GB": round(h2d / 1e9, 3), "d2h_GB": round(d2h / 1e9, 3),
                     "link_GB/s": round((h2d + d2h) / (ms * 1e-3) / 1e9, 1)}
        # the pipelined step: bundles of cells on two copy streams
        for nbundle in (4, 16):
            sph.sph_offload_step_async(plan, host, dev, ws, nbundle=nbundle, tuning=tuning)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                sph.sph_offload_step_async(plan, host, dev, ws, nbundle=nbundle, tuning=tuning)
            e1.record(stream)
            torch.cuda.synchronize()
            res[name][f"async{nbundle}_ms_per_step"] = round(e0.elapsed_time(e1) / reps, 3)
        log(f"offload {name}: {ms:.1f} ms/step, {res[name]}")
        del dev, host
        torch.cuda.empty_cache()
    # a plain pinned copy of the same volume, for the link's reference rate
    nb = 1 << 30
    hsrc = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
    dd = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dd.copy_(hsrc, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    dd.copy_(hsrc, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    res["pinned_copy_h2d_GB/s"] = round(nb / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    return res


def cpu_baseline(ps, store, budget_s, layout_name):
    """The oracle timed on the host: its interaction loops (FP64, OpenMP, the
    candidate-grid mode: every particle within the largest support visited,
    the same sums as its brute force) on sampled rows, all three loops, in
    interacting pairs per second; beside it the oracle's plain-C pack and
    unpack (per-loop form, one host thread) of the workload's first cells in
    GB/s of the same algorithmic bytes as the device figures."""
    import oracle

    f = ps.fields
    rho = store.get("rho").astype(np.float64)
    rdh = store.get("rho_dh").astype(np.float64)
    D = store.get("div_v").astype(np.float64)
    R = store.get("rot_v").astype(np.float64)
    rng = np.random.default_rng(0)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # grow the sample until one run takes at least half the budget (the oracle
    # converts its whole input on every call, so short runs are overhead) and
    # report that run
    nrow = 1024
    while True:
        rows = rng.choice(ps.n, nrow, replace=False)
        t0 = time.perf_counter()
        c = _oracle_rows(oracle, f, rho, rdh, D, R, rows)
        dt = time.perf_counter() - t0
        if dt >= 0.5 * budget_s or nrow >= ps.n:
            break
        nrow = int(min(ps.n, nrow * min(8.0, max(2.0, 0.8 * budget_s / dt))))
    out = {"value": c / dt, "unit": "pair interactions/s", "cores": cores, "kind": "oracle",
           "sample": f"{nrow} random particles of the workload, density+gradient+force, each summed over the "
                     f"particles of the oracle's candidate grid (FP64; the same sums as its brute force over "
                     f"all {ps.n}) ({dt:.1f} s)",
           "seconds": dt}
    out["host_pack_unpack"] = _oracle_pack_unpack(oracle, ps, sph_layout_index(layout_name))
    return out


def sph_layout_index(name):
    import oracle
    return oracle.LAYOUTS.index(name)


def _oracle_pack_unpack(oracle, ps, layout, target=1 << 20):
    """the oracle's pack and unpack of every loop (per-loop form: pack, then
    unpack of a result buffer) over the first cells holding about `target`
    particles, one host thread"""
    csum = np.cumsum(ps.cells["count"])
    k = int(min(len(csum), np.searchsorted(csum, target) + 1))
    n_sub = int(csum[k - 1])
    cells = np.ascontiguousarray(ps.cells[:k])
    host = oracle.HostStore(layout, n_sub)
    host.put_all({name: np.ascontiguousarray(v[:n_sub]) for name, v in ps.fields.items()})
    rng = np.random.default_rng(1)
    res = {L: rng.uniform(-1, 1, (oracle.RESULT_PLANES[L], oracle.round_slots(n_sub))).astype(np.float32)
           for L in range(3)}
    t0 = time.perf_counter()
    for L in range(3):
        oracle.pack_cells(host, L, cells)
        oracle.unpack_cells(host, L, res[L])
    dt = time.perf_counter() - t0
    nbytes = sum((PACK_BYTES[L] + UNPACK_BYTES[L]) * n_sub for L in range(3))
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"pack + unpack of the three loops over the first {k} cells ({n_sub} particles) of the "
                      f"workload, {oracle.LAYOUTS[layout]} store, per-loop form ({dt:.2f} s)",
            "seconds": dt}


def _oracle_rows(oracle, f, rho, rdh, D, R, rows):
    d = oracle.density(f["x"], f["mass"], f["h"], rows=rows, grid=True)
    g = oracle.gradient(f["x"], f["v"], f["mass"], f["h"], f["u"], rho, rows=rows, grid=True)
    fo = oracle.force(f["x"], f["v"], f["mass"], f["h"], f["u"], rho, rdh, D, R, f["alpha_v"], f["alpha_d"],
                      rows=rows, grid=True)
    return int(d["count"].sum() + g["count"].sum() + fo["count"].sum())


if __name__ == "__main__":
    main()
