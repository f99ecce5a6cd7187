"""Full-size workloads in the launch configuration the benchmark times
(batched form, default tuning, kernels without pair counts; the counting
kernels are checked too): sampled particles against the oracle, each loop
fed the GPU's previous-loop outputs.  256^3 Gresho on 32^3 cells and the 188^3
clustered set on its octree."""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

from gpuhelp import LOOP_OUT, compare_loop, device_store, log, oracle_loop, outputs, run_batched_loop

pytestmark = pytest.mark.gpu


def _run(k, nrows, layout, convert_to=None):
    log(f"building workload {k}")
    ps = inputs.make_config(k)
    log(f"n={ps.n} cells={len(ps.cells)} tasks={len(ps.tasks)} {inputs.cell_stats(ps.cells)}")
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, layout)
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(ps.n, nrows, replace=False))
    # the largest cells and the smallest supports are where errors concentrate
    big = int(np.argmax(ps.cells["count"]))
    rows = np.unique(np.r_[rows, ps.cells["first"][big] + np.arange(min(16, ps.cells["count"][big])),
                           np.argsort(ps.fields["h"])[:16]])
    eps = oracle.pack_resolution(ps.cells)
    prev = {}
    for loop in range(3):
        cnt = run_batched_loop(plan, st, loop, counts=True)
        gcnt = outputs(st, loop)
        run_batched_loop(plan, st, loop)  # without counts, as the benchmark times it
        g = outputs(st, loop)
        log(f"loop {loop}: oracle on {rows.size} rows")
        ref = oracle_loop(ps.fields, loop, prev, rows=rows, epsx=eps)
        errs = compare_loop(loop, g, ref, rows=rows)
        for k, e in compare_loop(loop, gcnt, ref, rows=rows).items():
            errs[k] = max(errs[k], e)
        log(f"loop {loop}: worst {max(errs.values()):.2e} {errs}")
        assert max(errs.values()) <= 1e-5, errs
        dc = np.abs(cnt[rows].astype(np.int64) - ref["count"])
        assert np.all(dc <= ref["band"]), (loop, int(dc.max()))
        for kk in LOOP_OUT[loop]:
            prev[kk] = g[kk].astype(np.float64)
    if convert_to is not None:
        # the whole store, outputs included, rewritten into another layout
        log(f"convert {sph.LAYOUTS[layout]} -> {sph.LAYOUTS[convert_to]} n={ps.n}")
        dst = sph.Store(convert_to, ps.n)
        sph.sph_store_convert(st, dst)
        for name in sph.FIELDS:
            assert st.get(name).tobytes() == dst.get(name).tobytes(), name
    plan.close()


def test_gresho256_sampled():
    _run(2, 96, sph.LAYOUTS.index("SAOS_SHARED"), convert_to=sph.LAYOUTS.index("SOA"))


def test_clustered188_sampled():
    _run(3, 96, sph.LAYOUTS.index("SOA"))
