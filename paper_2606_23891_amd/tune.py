"""Autotuner for the batched form's launch parameters.

For each loop it times the interaction kernel over candidate windows (the LDS
candidate buffer per wave) and persistent-grid sizes (blocks per CU), each loop
keeping its own, under each work distribution (static stride, one queue, per-XCD
queues; shared by the loops), and times pack + unpack over
waves per block; it keeps the fastest of each (median of a few HIP-event
timed repetitions on the device) and records them in a JSON cache keyed by
device name and workload signature.  ``bench.py --tuning auto`` reads the cache.

Usage: python -m paper_2606_23891_amd.tune [--config 2] [--grid 32] [--layout SAOS_SHARED]
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning_cache.json")

WINDOWS = {0: (128, 256, 512), 1: (128, 256, 512), 2: (128, 256)}
BLOCKS_PER_CU = (2, 4, 8, 16)
QUEUE = (2, 1, 0)
PACK_WAVES = (1, 2, 4, 8)


def device_key(props) -> str:
    """the tuning cache's device key: ISA name and compute-unit count (the
    marketing name is not reported under every tool, e.g. a profiler)"""
    arch = getattr(props, "gcnArchName", "") or props.name
    return f"{arch.split(':')[0]}-{props.multi_processor_count}cu"


def signature(ps, layout_name: str) -> str:
    st = ps.meta
    return f"cfg{st.get('config')}-n{ps.n}-cells{len(ps.cells)}-tasks{len(ps.tasks)}-{layout_name}"


def load(device: str, sig: str):
    if not os.path.exists(CACHE):
        return None
    try:
        data = json.load(open(CACHE))
    except (OSError, ValueError):
        return None
    return data.get(device, {}).get(sig)


def apply(tuning, entry: dict):
    for k, v in entry.items():
        if k in ("window", "blocks_per_loop"):
            arr = getattr(tuning, k)
            for i, w in enumerate(v):
                arr[i] = int(w)
        elif k in ("blocks_per_cu", "pack_waves", "queue", "pack_schedule"):
            setattr(tuning, k, int(v))
    return tuning


def _timed(fn, reps=3):
    import torch
    s = torch.cuda.current_stream()
    fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(plan, store, log=print):
    """Return (best sph_tuning fields as a dict, timings)."""
    import torch

    from . import sph

    ws = sph.interact_ws(plan)
    params = sph.default_params()
    best = {"window": [256, 256, 128], "blocks_per_cu": 8, "queue": 1, "pack_waves": 4}
    times = {}
    bufs = {L: sph.cell_buffers(plan, L) for L in range(3)}
    # make every loop's inputs valid: one plain pass through the three loops
    t = sph.default_tuning()
    for L in range(3):
        pack, res = bufs[L]
        sph.sph_pack_cells(plan, L, store, pack, t)
        sph.sph_interact_cells(plan, L, pack, res, ws, params=params, tuning=t)
        sph.sph_unpack_cells(plan, L, res, store, t)
    torch.cuda.synchronize()
    # pack / unpack waves per block (all loops together)
    pw_best, pw_t = None, None
    for pw in PACK_WAVES:
        t = sph.default_tuning()
        t.pack_waves = pw

        def run():
            for L in range(3):
                pack, res = bufs[L]
                sph.sph_pack_cells(plan, L, store, pack, t)
                sph.sph_unpack_cells(plan, L, res, store, t)
        ms = _timed(run)
        times[f"pack_unpack_waves{pw}"] = ms
        log(f"pack+unpack waves={pw}: {ms:.3f} ms")
        if pw_t is None or ms < pw_t:
            pw_best, pw_t = pw, ms
    best["pack_waves"] = pw_best
    # loop fission of the conversions: the fused kernels or one of the split
    # schedules, whichever moves the layout's fields fastest
    ps_best, ps_t = 0, None
    for sname, sched in sph.SCHEDULES.items():
        t = sph.default_tuning()
        t.pack_waves, t.pack_schedule = pw_best, sched

        def run():
            for L in range(3):
                pack, res = bufs[L]
                sph.sph_pack_cells(plan, L, store, pack, t)
                sph.sph_unpack_cells(plan, L, res, store, t)
        ms = _timed(run)
        times[f"pack_unpack_{sname}"] = ms
        log(f"pack+unpack {sname}: {ms:.3f} ms")
        if ps_t is None or ms < ps_t:
            ps_best, ps_t = sched, ms
    best["pack_schedule"] = ps_best
    # interaction kernels: each loop takes its own window and grid size; the
    # queue mode is shared, chosen on the sum of the loops' best times
    totals = {}
    for q in QUEUE:
        tot, wins, bpcs = 0.0, [], []
        for L in range(3):
            pack, res = bufs[L]
            sph.sph_pack_cells(plan, L, store, pack)
            bk, bt = None, None
            for bpc, w in itertools.product(BLOCKS_PER_CU, WINDOWS[L]):
                t = sph.default_tuning()
                t.blocks_per_cu, t.queue = bpc, q
                t.window[L] = w
                ms = _timed(lambda: sph.sph_interact_cells(plan, L, pack, res, ws, params=params, tuning=t))
                times[f"loop{L}_bpc{bpc}_q{q}_w{w}"] = ms
                if bt is None or ms < bt:
                    bk, bt = (bpc, w), ms
            tot += bt
            bpcs.append(bk[0])
            wins.append(bk[1])
        totals[q] = (tot, wins, bpcs)
        log(f"queue={q}: {tot:.3f} ms (windows {wins}, blocks/CU {bpcs})")
    q, (tot, wins, bpcs) = min(totals.items(), key=lambda kv: kv[1][0])
    best.update(blocks_per_cu=bpcs[2], blocks_per_loop=bpcs, queue=q, window=wins)
    return best, times


def choose_layout(plan, fields, layouts=None, tuning=None, log=print):
    """Time pack + unpack of the three loops (batched form) for each candidate
    store layout on the same particles and return (fastest layout name,
    {layout: ms}): the measured choice among the decompositions (a store is
    then moved into it with sph_store_convert)."""
    import torch

    from . import sph

    names = layouts or sph.LAYOUTS
    bufs = {L: sph.cell_buffers(plan, L) for L in range(3)}
    times = {}
    for name in names:
        st = sph.Store(sph.LAYOUTS.index(name), plan.n)
        st.put_all(fields)

        def run():
            for L in range(3):
                pack, res = bufs[L]
                sph.sph_pack_cells(plan, L, st, pack, tuning)
                sph.sph_unpack_cells(plan, L, res, st, tuning)
        times[name] = _timed(run)
        log(f"layout {name}: pack+unpack {times[name]:.3f} ms")
        del st
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    return best, times


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--grid", type=int, default=None)
    ap.add_argument("--n-side", type=int, default=None)
    ap.add_argument("--layout", default="SAOS_SHARED")
    ap.add_argument("--choose-layout", action="store_true",
                    help="only time pack + unpack per store layout and print the fastest")
    a = ap.parse_args()
    import torch

    from . import inputs, sph

    kw = {}
    if a.grid:
        kw["grid"] = a.grid
    if a.n_side:
        kw["n_side"] = a.n_side
    ps = inputs.make_config(a.config, **kw)
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    if a.choose_layout:
        best, times = choose_layout(plan, ps.fields)
        print(json.dumps({"best_layout": best, "pack_unpack_ms": times}))
        return
    store = sph.Store(sph.LAYOUTS.index(a.layout), ps.n)
    store.put_all(ps.fields)
    dev = device_key(torch.cuda.get_device_properties(0))
    sig = signature(ps, a.layout)
    log = lambda m: print(f"[tune {time.strftime('%H:%M:%S')}] {m}", file=sys.stderr, flush=True)
    best, times = tune(plan, store, log)
    data = {}
    if os.path.exists(CACHE):
        try:
            data = json.load(open(CACHE))
        except ValueError:
            data = {}
    data.setdefault(dev, {})[sig] = best
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    print(json.dumps({"device": dev, "workload": sig, "best": best, "times_ms": times}))


if __name__ == "__main__":
    main()
