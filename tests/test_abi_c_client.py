"""The C-ABI from plain C: a C99 client (tests/c_client/sph_abi_client.c)
that includes only include/sph.h and the HIP runtime's memory calls.

On the CPU: the header and client compile under gcc -std=c99 -pedantic
-Werror; the client's view of the layout, field and packed-record tables
matches the oracle's own tables and the Python binding's; invalid arguments
fail with the documented codes before any device is touched.  On the GPU: the
client's batched step, and its per-task pack -> interact -> unpack calls, over
a particle set read from a file give outputs bit for bit equal to the same
calls through the Python binding, and within the parity tolerance of the
oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_client"))
import build_client  # noqa: E402

OUT_FIELDS = [("rho", 1), ("rho_dh", 1), ("wcount", 1), ("div_v", 1), ("rot_v", 3), ("lap_u", 1), ("v_sig", 1),
              ("a", 3), ("u_dt", 1)]


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    return build_client.build(str(tmp_path_factory.mktemp("cclient") / "sph_abi_client"))


def _tables(binary):
    r = subprocess.run([binary, "tables"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    return [ln.split() for ln in r.stdout.splitlines()]


def test_client_tables_match_oracle_and_binding(client):
    rows = _tables(client)
    status = {int(r[1]): " ".join(r[2:]) for r in rows if r[0] == "status"}
    assert status[0] == "ok" and len(status) == 7
    layouts = {int(r[1]): [int(v) for v in r[3:]] for r in rows if r[0] == "layout"}
    assert all(int(r[2]) == len(r) - 3 for r in rows if r[0] == "layout")
    assert sorted(layouts) == list(range(10))
    for lay, sub_bytes in layouts.items():
        assert sub_bytes == list(oracle.layout_info(lay)) == list(sph.sph_layout_info(lay)), lay
    fields = [tuple(int(v) for v in r[1:]) for r in rows if r[0] == "field"]
    n_comp = sum(sph.sph_field_info(f)[0] for f in range(len(sph.FIELDS)))
    assert len(fields) == 10 * n_comp
    for lay, fid, c, sub, off, stride in fields:
        assert (sub, off, stride) == tuple(oracle.field_location(lay, fid, c)), (lay, fid, c)
    packs = {int(r[1]): (int(r[2]), tuple(int(v) for v in r[3:])) for r in rows if r[0] == "pack"}
    for loop in range(3):
        assert packs[loop] == (oracle.RESULT_PLANES[loop], tuple(oracle.PACK_PLANES[loop]))
    tun = [int(v) for v in next(r for r in rows if r[0] == "tuning")[1:]]
    t = sph.default_tuning()
    assert tun == [t.blocks_per_cu, *t.window, t.pack_waves, t.queue, *t.blocks_per_loop, t.pack_schedule]
    invalid = {r[1]: int(r[2]) for r in rows if r[0] == "invalid"}
    assert invalid == {"plan_null_cells": -1, "plan_negative_n": -1, "plan_task_cell": -4, "layout": -2,
                       "plan_out": -1}


def _write_input(path, ps, layout):
    f = ps.fields
    with open(path, "wb") as fh:
        fh.write(np.array([ps.n], "<i8").tobytes())
        fh.write(np.array([len(ps.cells), len(ps.tasks), layout, 0], "<i4").tobytes())
        fh.write(np.ascontiguousarray(ps.cells).tobytes())
        fh.write(np.ascontiguousarray(ps.tasks).tobytes())
        fh.write(np.ascontiguousarray(f["x"], "<f8").tobytes())
        fh.write(np.ascontiguousarray(f["v"], "<f4").tobytes())
        for k in ("mass", "h", "u", "alpha_v", "alpha_d"):
            fh.write(np.ascontiguousarray(f[k], "<f4").tobytes())


def _read_output(path, n):
    raw = np.fromfile(path, "<f4")
    out, o = {}, 0
    for name, nc in OUT_FIELDS:
        a = raw[o:o + n * nc]
        out[name] = a.reshape(n, nc) if nc > 1 else a
        o += n * nc
    assert o == raw.size
    return out


BUNDLE = 8


@pytest.mark.gpu
@pytest.mark.parametrize("mode,layout", [("step", "SAOS_SHARED"), ("step", "AOS"), ("step", "SOA"),
                                         ("per_task", "SAOS_SHARED"), ("per_task", "SOA")])
def test_client_step_matches_binding_and_oracle(mode, layout, tmp_path):
    """step: sph_step_batched; per_task: the five per-task calls (pack,
    density / gradient / force, unpack) over bundles of 8 tasks"""
    import torch

    from gpuhelp import LOOP_OUT, compare_loop, device_store, log, oracle_loop, run_per_task
    binary = build_client.BIN
    assert os.path.exists(binary), "the C client is built by __graft_entry__.build()"
    ps = inputs.make_config(1, n_side=24, grid=4)   # 216 particles per cell: ragged tiles
    lay = sph.LAYOUTS.index(layout)
    _write_input(tmp_path / "in.bin", ps, lay)
    log(f"C client {mode} {layout} n={ps.n} tasks={len(ps.tasks)}")
    args = [binary, mode, str(tmp_path / "in.bin"), str(tmp_path / "out.bin")]
    if mode == "per_task":
        args.append(str(BUNDLE))
    r = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = _read_output(tmp_path / "out.bin", ps.n)
    # the same through the Python binding: bit for bit
    plan = sph.Plan(ps.cells, ps.tasks, ps.n)
    st = device_store(ps, lay)
    if mode == "step":
        ws = torch.zeros(sph.sph_batched_ws_bytes(plan), dtype=torch.uint8, device="cuda")
        sph.sph_step_batched(plan, st, ws)
    else:
        for loop in range(3):
            run_per_task(plan, st, loop, len(ps.tasks), bundle=BUNDLE)
    torch.cuda.synchronize()
    for name, _ in OUT_FIELDS:
        assert st.get(name).tobytes() == got[name].tobytes(), name
    # and against the oracle, each loop fed the client's previous-loop outputs
    eps = oracle.pack_resolution(ps.cells)
    prev = {}
    for loop in range(3):
        ref = oracle_loop(ps.fields, loop, prev, epsx=eps, grid=True)
        errs = compare_loop(loop, {k: got[k] for k in LOOP_OUT[loop]}, ref)
        log(f"C client {mode} {layout} loop {loop}: worst {max(errs.values()):.2e}")
        assert max(errs.values()) <= 1e-5, errs
        for k in LOOP_OUT[loop]:
            prev[k] = got[k].astype(np.float64)
    plan.close()
