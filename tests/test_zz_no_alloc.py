"""The allocation-free batched step (sph_step_batched_noalloc, workspace in the
library's static per-device scratch) against sph_step_batched with a caller
workspace: the same kernels, so the stores must agree byte for byte.  Two
calls in a row, the second on a smaller set (the scratch keeps the first
call's contents), then a third call on the first set again; a plan whose
workspace exceeds the scratch is refused before anything is written."""
import numpy as np
import pytest

from paper_2606_23891_amd import inputs, sph

from gpuhelp import device_store, log

pytestmark = pytest.mark.gpu


def _reference(ps, layout):
    import torch
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, layout)
    ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
    sph.sph_step_batched(plan, st, ws)
    torch.cuda.synchronize()
    out = st.raw()
    plan.close()
    return out


def _noalloc(ps, layout):
    import torch
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    assert sph.sph_batched_ws_bytes(plan) <= sph.NOALLOC_SCRATCH_BYTES
    st = device_store(ps, layout)
    sph.sph_step_batched_noalloc(plan, st)
    torch.cuda.synchronize()
    out = st.raw()
    plan.close()
    return out


def test_noalloc_step_matches_workspace_step():
    lay = sph.LAYOUTS.index("SAOS_SHARED")
    big = inputs.make_config(1, n_side=32)      # 32 768 particles
    small = inputs.make_config(4, n_side=16)    # 4 096 particles
    for name, ps in (("32^3 Gresho", big), ("16^3 adjoint lattice", small), ("32^3 Gresho again", big)):
        log(f"noalloc step on {name}: n={ps.n}")
        assert _noalloc(ps, lay) == _reference(ps, lay), name


def test_noalloc_refuses_oversize_plan():
    import torch
    ps = inputs.make_config(0, n_side=84, grid=16)   # 592 704 particles: workspace beyond 64 MiB
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    need = sph.sph_batched_ws_bytes(plan)
    log(f"oversize plan: n={ps.n} needs {need} bytes")
    assert need > sph.NOALLOC_SCRATCH_BYTES
    st = device_store(ps, sph.LAYOUTS.index("SOA"))
    before = st.raw()
    with pytest.raises(sph.SphError, match="static scratch"):
        sph.sph_step_batched_noalloc(plan, st)
    torch.cuda.synchronize()
    assert st.raw() == before
    plan.close()
