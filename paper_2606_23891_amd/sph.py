"""Thin ctypes binding of libsph (argument marshalling only).

Every function here forwards to the C entry point of the same name declared in
``include/sph.h``; all arithmetic runs in the HIP kernels of the library.
Device memory and streams come from PyTorch (ROCm): buffers are torch tensors
passed by ``data_ptr()``, streams by ``torch.cuda.current_stream().cuda_stream``.
The library must exist (built by ``python -m paper_2606_23891_amd.build``);
loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

DENSITY, GRADIENT, FORCE = 0, 1, 2
LOOPS = (DENSITY, GRADIENT, FORCE)
LAYOUTS = ["AOS", "AOS_RANDOM", "SAOS_GRAD", "SAOS_FORCE", "SAOS_SHARED", "SAOS_GRAD_TYPE",
           "SAOS_FORCE_TYPE", "SAOS_SHARED_TYPE", "SOA", "SAOS_SHARED_REPL"]
FIELDS = ["x", "v", "a", "mass", "h", "u", "u_dt", "rho", "rho_dh", "wcount", "div_v", "rot_v",
          "lap_u", "v_sig", "alpha_v", "alpha_d", "time_bin", "id", "cold"]
FIELD_ID = {n: i for i, n in enumerate(FIELDS)}
MAX_SUB = 32
STATUS = {0: "SPH_OK", -1: "SPH_E_ARG", -2: "SPH_E_LAYOUT", -3: "SPH_E_CAPACITY", -4: "SPH_E_PLAN",
          -5: "SPH_E_HIP", -6: "SPH_E_UNSUPPORTED"}


class sph_store(C.Structure):
    _fields_ = [("layout", C.c_int32), ("nsub", C.c_int32), ("n", C.c_int64),
                ("sub", C.c_void_p * MAX_SUB)]


class sph_params(C.Structure):
    _fields_ = [("gamma_ad", C.c_float), ("beta_visc", C.c_float), ("balsara_eps", C.c_float),
                ("pad", C.c_float)]


class sph_tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("window", C.c_int32 * 3), ("pack_waves", C.c_int32),
                ("queue", C.c_int32), ("blocks_per_loop", C.c_int32 * 3), ("pack_schedule", C.c_int32)]


class sph_plan_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("ncell", C.c_int32), ("ntask", C.c_int32), ("nslot", C.c_int64),
                ("nchunk", C.c_int64), ("ntile", C.c_int32), ("max_cell", C.c_int32),
                ("max_nbr", C.c_int32), ("batched_ok", C.c_int32), ("mixed_widths", C.c_int32),
                ("pad", C.c_int32)]


class SphError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


_lib = None
vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
_SIGS = {
    "sph_status_str": ([i32], C.c_char_p),
    "sph_last_error": ([], C.c_char_p),
    "sph_layout_info": ([i32, C.POINTER(i32), C.POINTER(sz)], i32),
    "sph_field_location": ([i32, i32, i32, C.POINTER(i32), C.POINTER(sz), C.POINTER(sz)], i32),
    "sph_x_replicas": ([i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(sz)], i32),
    "sph_field_info": ([i32, C.POINTER(i32), C.POINTER(i32)], i32),
    "sph_pack_layout": ([i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)], i32),
    "sph_fission_passes": ([i32, i32, i32, C.POINTER(i32), C.POINTER(C.c_uint32), C.POINTER(i32),
                            C.POINTER(C.c_uint32)], i32),
    "sph_store_put": ([vp, i32, vp, vp], i32),
    "sph_store_get": ([vp, i32, vp, vp], i32),
    "sph_store_convert": ([vp, vp, vp], i32),
    "sph_plan_create": ([vp, i32, vp, i32, i64, C.POINTER(vp)], i32),
    "sph_plan_destroy": ([vp], None),
    "sph_plan_get_info": ([vp, vp], i32),
    "sph_plan_buffer_bytes": ([vp, i32, i32, i32, C.POINTER(i64), C.POINTER(sz), C.POINTER(sz)], i32),
    "sph_plan_cell_reach": ([vp, vp], i32),
    "sph_zero_outputs": ([vp, i32, vp, vp], i32),
    "sph_pack": ([vp, i32, vp, i32, i32, vp, sz, vp], i32),
    "sph_density": ([vp, vp, sz, i32, i32, vp, vp, sz, vp, vp], i32),
    "sph_gradient": ([vp, vp, sz, i32, i32, vp, vp, sz, vp, vp], i32),
    "sph_force": ([vp, vp, sz, i32, i32, vp, vp, sz, vp, vp], i32),
    "sph_unpack": ([vp, i32, vp, sz, i32, i32, vp, vp], i32),
    "sph_run_per_task": ([vp, i32, vp, i32, i32, i32, vp, vp, sz, vp, sz, vp], i32),
    "sph_plan_task_max_bytes": ([vp, i32, C.POINTER(sz), C.POINTER(sz)], i32),
    "sph_tuning_default": ([vp], None),
    "sph_batched_ws_bytes": ([vp, C.POINTER(sz)], i32),
    "sph_pack_cells": ([vp, i32, vp, vp, sz, vp, vp], i32),
    "sph_interact_ws_bytes": ([vp, i32, C.POINTER(sz)], i32),
    "sph_interact_cells": ([vp, i32, vp, sz, vp, vp, vp, sz, vp, vp, sz, vp], i32),
    "sph_unpack_cells": ([vp, i32, vp, sz, vp, vp, vp], i32),
    "sph_step_batched": ([vp, vp, vp, vp, vp, sz, vp], i32),
    "sph_step_batched_noalloc": ([vp, vp, vp, vp, vp], i32),
    "sph_step_pack": ([vp, i32, vp, vp, vp, vp, sz, vp], i32),
    "sph_step_interact": ([vp, i32, vp, vp, vp, sz, vp], i32),
    "sph_step_writeback": ([vp, vp, vp, vp, sz, vp], i32),
    "sph_step_output_writers": ([i32, vp], i32),
    "sph_integrate_ws_bytes": ([vp, C.POINTER(sz)], i32),
    "sph_kick": ([vp, C.c_float, vp], i32),
    "sph_drift": ([vp, vp, C.c_double, vp, sz, C.POINTER(C.c_double), C.POINTER(C.c_float), vp], i32),
    "sph_cfl_dt": ([vp, vp, C.c_float, vp, sz, C.POINTER(C.c_float), vp], i32),
    "sph_step_kdk": ([vp, vp, vp, vp, C.c_float, vp, sz, C.POINTER(i32), vp], i32),
    "sph_h_iterate_ws_bytes": ([vp, C.POINTER(sz)], i32),
    "sph_h_iterate": ([vp, vp, vp, vp, C.c_float, C.c_float, i32, vp, sz, C.POINTER(i32), C.POINTER(i64), vp],
                      i32),
    "sph_graph_capture": ([vp, vp, vp, vp, vp, sz, C.POINTER(vp)], i32),
    "sph_graph_launch": ([vp, vp], i32),
    "sph_graph_destroy": ([vp], None),
    "sph_offload_bytes": ([i32, i32, i64, C.POINTER(sz), C.POINTER(sz)], i32),
    "sph_offload_step": ([vp, vp, vp, vp, vp, vp, sz, vp], i32),
    "sph_offload_step_async": ([vp, vp, vp, vp, vp, i32, vp, sz, vp], i32),
    "sph_adjoint_ws_bytes": ([vp, C.POINTER(sz)], i32),
    "sph_adjoint_forward": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp], i32),
    "sph_force_adjoint": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp], i32),
    "sph_density_adjoint": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp], i32),
}


def lib():
    """Load libsph.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_23891_amd.build`")
    # torch carries its own HIP runtime under the same soname as the one the
    # library links (libamdhip64.so.7); whichever is loaded first serves the
    # whole process, and torch does not run on another runtime.  Load torch's
    # first, so that the library and torch share it.
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status: int, where: str):
    if status != 0:
        raise SphError(status, where, lib().sph_last_error().decode())


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def default_params() -> sph_params:
    return sph_params(5.0 / 3.0, 3.0, 1e-4, 0.0)


def default_tuning() -> sph_tuning:
    t = sph_tuning()
    lib().sph_tuning_default(C.byref(t))
    return t


# ---------------------------------------------------------------------------
# host-only queries
# ---------------------------------------------------------------------------
def sph_layout_info(layout: int):
    n = i32()
    sb = (sz * MAX_SUB)()
    _check(lib().sph_layout_info(layout, C.byref(n), sb), "sph_layout_info")
    return [int(sb[i]) for i in range(n.value)]


def sph_field_location(layout: int, field: int, comp: int):
    s, o, st = i32(), sz(), sz()
    _check(lib().sph_field_location(layout, field, comp, C.byref(s), C.byref(o), C.byref(st)),
           "sph_field_location")
    return s.value, o.value, st.value


def sph_x_replicas(layout: int):
    """[(substruct, byte offset of component 0)] of the copies of x beyond the primary one"""
    n = i32()
    sb = (i32 * 3)()
    of = (sz * 3)()
    _check(lib().sph_x_replicas(layout, C.byref(n), sb, of), "sph_x_replicas")
    return [(sb[r], of[r]) for r in range(n.value)]


def sph_field_info(field: int):
    n, b = i32(), i32()
    _check(lib().sph_field_info(field, C.byref(n), C.byref(b)), "sph_field_info")
    return n.value, b.value


def sph_pack_layout(loop: int):
    n, rp = i32(), i32()
    pf = (i32 * 5)()
    _check(lib().sph_pack_layout(loop, C.byref(n), pf, C.byref(rp)), "sph_pack_layout")
    return [pf[i] for i in range(n.value)], rp.value


MAX_PASSES = 32
SCHEDULES = {"by_particle": 0, "by_struct": 1, "by_element": 2, "by_type": 3, "by_struct_and_type": 4}


def sph_fission_passes(layout: int, loop: int, schedule: int):
    """(pack masks, unpack masks) of the kernels a fissioned pack / unpack runs."""
    npk, nun = i32(), i32()
    pm, um = (C.c_uint32 * MAX_PASSES)(), (C.c_uint32 * MAX_PASSES)()
    _check(lib().sph_fission_passes(layout, loop, schedule, C.byref(npk), pm, C.byref(nun), um),
           "sph_fission_passes")
    return [int(pm[i]) for i in range(npk.value)], [int(um[i]) for i in range(nun.value)]


# ---------------------------------------------------------------------------
# device objects
# ---------------------------------------------------------------------------
class Store:
    """A particle store of one layout, substructs held as torch uint8 tensors
    (device memory, or pinned host memory with device="pinned")."""

    def __init__(self, layout: int, n: int, device="cuda"):
        import torch
        self.layout, self.n = layout, n
        self.sub_bytes = sph_layout_info(layout)
        if device == "pinned":
            self.subs = [torch.zeros(max(1, n * b) + 256, dtype=torch.uint8, pin_memory=True) for b in self.sub_bytes]
            self.subs = [_aligned_view(t, max(1, n * b)) for t, b in zip(self.subs, self.sub_bytes)]
        else:
            self.subs = [torch.zeros(max(1, n * b), dtype=torch.uint8, device=device) for b in self.sub_bytes]
        self.c = sph_store()
        self.c.layout = layout
        self.c.nsub = len(self.subs)
        self.c.n = n
        for i, t in enumerate(self.subs):
            self.c.sub[i] = t.data_ptr()

    @property
    def ref(self):
        return C.byref(self.c)

    def put(self, name: str, arr, stream=None):
        import torch
        t = torch.as_tensor(np.ascontiguousarray(arr)).to(self.subs[0].device)
        sph_store_put(self, FIELD_ID[name], t, stream)

    def get(self, name: str, stream=None) -> np.ndarray:
        import torch
        if not self.subs[0].is_cuda:
            raise RuntimeError("field access of a host store: use sph_store_get on a device copy")
        nc, cb = sph_field_info(FIELD_ID[name])
        dt = {("x", 8): torch.float64, ("id", 8): torch.int64, ("cold", 8): torch.int64}.get(
            (name, cb), {4: torch.float32, 1: torch.int8}.get(cb))
        t = torch.empty((self.n, nc) if nc > 1 else (self.n,), dtype=dt, device=self.subs[0].device)
        sph_store_get(self, FIELD_ID[name], t, stream)
        torch.cuda.synchronize()
        out = t.cpu().numpy()
        return out.view(np.uint64) if name == "cold" else out

    def put_all(self, fields: Dict[str, np.ndarray]):
        for k, v in fields.items():
            if k == "cold":
                v = np.ascontiguousarray(v).view(np.int64)
            self.put(k, v)

    def raw(self) -> bytes:
        import torch
        torch.cuda.synchronize()
        return b"".join(t[: self.n * b].cpu().numpy().tobytes() for t, b in zip(self.subs, self.sub_bytes))


def _aligned_view(t, nbytes: int):
    """a 256-byte aligned view of nbytes inside the host tensor t"""
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def sph_plan_cell_reach(plan) -> np.ndarray:
    out = np.zeros(len(plan.cells), np.float64)
    _check(lib().sph_plan_cell_reach(_h(plan), out.ctypes.data if out.size else None), "sph_plan_cell_reach")
    return out


class Plan:
    """Cells and tasks of one step, uploaded once."""

    def __init__(self, cells: np.ndarray, tasks: np.ndarray, n: int):
        self.cells = np.ascontiguousarray(cells)
        self.tasks = np.ascontiguousarray(tasks)
        assert self.cells.dtype.itemsize == 48 and self.tasks.dtype.itemsize == 40
        self.ptr = sph_plan_create(self.cells, self.tasks, n)
        self.n = n

    def info(self) -> sph_plan_info:
        return sph_plan_get_info(self)

    def buffer_bytes(self, loop: int, t0: int, t1: int):
        return sph_plan_buffer_bytes(self, loop, t0, t1)

    def cell_reach(self) -> np.ndarray:
        return sph_plan_cell_reach(self)

    def close(self):
        if self.ptr:
            lib().sph_plan_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _h(x):
    return x.ptr if isinstance(x, Plan) else x


def _s(x):
    return x.ref if isinstance(x, Store) else x


def sph_store_put(store, field: int, src, stream=None):
    _check(lib().sph_store_put(_s(store), field, _ptr(src), _stream(stream)), "sph_store_put")


def sph_store_get(store, field: int, dst, stream=None):
    _check(lib().sph_store_get(_s(store), field, _ptr(dst), _stream(stream)), "sph_store_get")


def sph_store_convert(src, dst, stream=None):
    """every member of every particle of src into dst (another layout's store)"""
    _check(lib().sph_store_convert(_s(src), _s(dst), _stream(stream)), "sph_store_convert")


def sph_plan_create(cells: np.ndarray, tasks: np.ndarray, n: int):
    out = vp()
    _check(lib().sph_plan_create(cells.ctypes.data if cells.size else None, cells.size,
                                 tasks.ctypes.data if tasks.size else None, tasks.size, n, C.byref(out)),
           "sph_plan_create")
    return out.value


def sph_plan_get_info(plan) -> sph_plan_info:
    info = sph_plan_info()
    _check(lib().sph_plan_get_info(_h(plan), C.byref(info)), "sph_plan_get_info")
    return info


def sph_plan_buffer_bytes(plan, loop: int, t0: int, t1: int):
    ns, pb, rb = i64(), sz(), sz()
    _check(lib().sph_plan_buffer_bytes(_h(plan), loop, t0, t1, C.byref(ns), C.byref(pb), C.byref(rb)),
           "sph_plan_buffer_bytes")
    return ns.value, pb.value, rb.value


def sph_zero_outputs(plan, loop: int, store, stream=None):
    _check(lib().sph_zero_outputs(_h(plan), loop, _s(store), _stream(stream)), "sph_zero_outputs")


def sph_pack(plan, loop: int, store, t0: int, t1: int, buf, stream=None):
    _check(lib().sph_pack(_h(plan), loop, _s(store), t0, t1, _ptr(buf), _nbytes(buf), _stream(stream)),
           "sph_pack")


def _nbytes(t) -> int:
    if t is None:
        return 0
    return t.numel() * t.element_size()


def _interact(name, plan, buf, t0, t1, params, res, counts, stream):
    fn = getattr(lib(), name)
    p = params if params is not None else default_params()
    _check(fn(_h(plan), _ptr(buf), _nbytes(buf), t0, t1, C.byref(p), _ptr(res), _nbytes(res), _ptr(counts),
              _stream(stream)), name)


def sph_density(plan, buf, t0, t1, res, params=None, counts=None, stream=None):
    _interact("sph_density", plan, buf, t0, t1, params, res, counts, stream)


def sph_gradient(plan, buf, t0, t1, res, params=None, counts=None, stream=None):
    _interact("sph_gradient", plan, buf, t0, t1, params, res, counts, stream)


def sph_force(plan, buf, t0, t1, res, params=None, counts=None, stream=None):
    _interact("sph_force", plan, buf, t0, t1, params, res, counts, stream)


INTERACT = {DENSITY: sph_density, GRADIENT: sph_gradient, FORCE: sph_force}


def sph_unpack(plan, loop: int, res, t0: int, t1: int, store, stream=None):
    _check(lib().sph_unpack(_h(plan), loop, _ptr(res), _nbytes(res), t0, t1, _s(store), _stream(stream)),
           "sph_unpack")


def sph_plan_task_max_bytes(plan, loop: int):
    pb, rb = sz(), sz()
    _check(lib().sph_plan_task_max_bytes(_h(plan), loop, C.byref(pb), C.byref(rb)), "sph_plan_task_max_bytes")
    return pb.value, rb.value


def sph_run_per_task(plan, loop: int, store, t0: int, t1: int, pack, res, zero_first=True, params=None,
                     stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_run_per_task(_h(plan), loop, _s(store), t0, t1, 1 if zero_first else 0, C.byref(p),
                                  _ptr(pack), _nbytes(pack), _ptr(res), _nbytes(res), _stream(stream)),
           "sph_run_per_task")


def sph_batched_ws_bytes(plan) -> int:
    b = sz()
    _check(lib().sph_batched_ws_bytes(_h(plan), C.byref(b)), "sph_batched_ws_bytes")
    return b.value


def sph_pack_cells(plan, loop: int, store, buf, tuning=None, stream=None):
    _check(lib().sph_pack_cells(_h(plan), loop, _s(store), _ptr(buf), _nbytes(buf),
                                C.byref(tuning) if tuning else None, _stream(stream)), "sph_pack_cells")


def sph_interact_ws_bytes(plan, loop: int) -> int:
    b = sz()
    _check(lib().sph_interact_ws_bytes(_h(plan), loop, C.byref(b)), "sph_interact_ws_bytes")
    return b.value


def sph_interact_cells(plan, loop: int, buf, res, ws, params=None, tuning=None, counts=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_interact_cells(_h(plan), loop, _ptr(buf), _nbytes(buf), C.byref(p),
                                    C.byref(tuning) if tuning else None, _ptr(res), _nbytes(res), _ptr(counts),
                                    _ptr(ws), _nbytes(ws), _stream(stream)), "sph_interact_cells")


def sph_unpack_cells(plan, loop: int, res, store, tuning=None, stream=None):
    _check(lib().sph_unpack_cells(_h(plan), loop, _ptr(res), _nbytes(res), _s(store),
                                  C.byref(tuning) if tuning else None, _stream(stream)), "sph_unpack_cells")


def sph_integrate_ws_bytes(plan) -> int:
    b = sz()
    _check(lib().sph_integrate_ws_bytes(_h(plan), C.byref(b)), "sph_integrate_ws_bytes")
    return b.value


def sph_kick(store, dt: float, stream=None):
    _check(lib().sph_kick(_s(store), float(dt), _stream(stream)), "sph_kick")


def sph_drift(plan, store, dt: float, ws, stream=None, report=True):
    """x += v dt; returns (largest distance outside a cell, largest h) when report"""
    mo, mh = C.c_double(), C.c_float()
    _check(lib().sph_drift(_h(plan), _s(store), float(dt), _ptr(ws), _nbytes(ws),
                           C.byref(mo) if report else None, C.byref(mh) if report else None, _stream(stream)),
           "sph_drift")
    return (mo.value, mh.value) if report else None


def sph_cfl_dt(plan, store, ws, cfl: float = 0.1, stream=None) -> float:
    dt = C.c_float()
    _check(lib().sph_cfl_dt(_h(plan), _s(store), float(cfl), _ptr(ws), _nbytes(ws), C.byref(dt),
                            _stream(stream)), "sph_cfl_dt")
    return dt.value


def kdk_ws_bytes(plan) -> int:
    """workspace of sph_step_kdk: the batched step's, rounded to 256, then the integrator's"""
    return (sph_batched_ws_bytes(plan) + 255) // 256 * 256 + sph_integrate_ws_bytes(plan)


def sph_step_kdk(plan, store, ws, dt: float, params=None, tuning=None, stream=None):
    """one kick-drift-kick step; returns 1 when the plan must be rebuilt (raises
    SphError then, with the status SPH_E_PLAN, after the drift)"""
    p = params if params is not None else default_params()
    rb = i32()
    _check(lib().sph_step_kdk(_h(plan), _s(store), C.byref(p), C.byref(tuning) if tuning else None, float(dt),
                              _ptr(ws), _nbytes(ws), C.byref(rb), _stream(stream)), "sph_step_kdk")
    return rb.value


def sph_h_iterate_ws_bytes(plan) -> int:
    b = sz()
    _check(lib().sph_h_iterate_ws_bytes(_h(plan), C.byref(b)), "sph_h_iterate_ws_bytes")
    return b.value


def sph_h_iterate(plan, store, ws, eta=1.2348, tol=1e-4, max_iter=30, params=None, tuning=None, stream=None):
    """Smoothing-length iteration; returns (passes run, particles still moving)."""
    p = params if params is not None else default_params()
    it, un = i32(), i64()
    _check(lib().sph_h_iterate(_h(plan), _s(store), C.byref(p), C.byref(tuning) if tuning else None,
                               float(eta), float(tol), int(max_iter), _ptr(ws), _nbytes(ws), C.byref(it),
                               C.byref(un), _stream(stream)), "sph_h_iterate")
    return it.value, un.value


def sph_step_batched(plan, store, ws, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_step_batched(_h(plan), _s(store), C.byref(p), C.byref(tuning) if tuning else None,
                                  _ptr(ws), _nbytes(ws), _stream(stream)), "sph_step_batched")


def sph_step_pack(plan, loop, store, ws, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_step_pack(_h(plan), loop, _s(store), C.byref(p), C.byref(tuning) if tuning else None,
                               _ptr(ws), _nbytes(ws), _stream(stream)), "sph_step_pack")


def sph_step_interact(plan, loop, ws, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_step_interact(_h(plan), loop, C.byref(p), C.byref(tuning) if tuning else None,
                                   _ptr(ws), _nbytes(ws), _stream(stream)), "sph_step_interact")


def sph_step_writeback(plan, store, ws, tuning=None, stream=None):
    _check(lib().sph_step_writeback(_h(plan), _s(store), C.byref(tuning) if tuning else None, _ptr(ws),
                                    _nbytes(ws), _stream(stream)), "sph_step_writeback")


STEP_OUTPUTS = [("rho", 0), ("rho_dh", 0), ("wcount", 0), ("div_v", 0), ("rot_v", 0), ("rot_v", 1),
                ("rot_v", 2), ("lap_u", 0), ("v_sig", 0), ("a", 0), ("a", 1), ("a", 2), ("u_dt", 0)]


def sph_step_output_writers(layout: int):
    """per step output (STEP_OUTPUTS order): 1 / 2 = stored by that loop's pack, 3 = by the write-back"""
    w = (i32 * 13)()
    _check(lib().sph_step_output_writers(layout, w), "sph_step_output_writers")
    return list(w)


NOALLOC_SCRATCH_BYTES = 64 << 20   # SPH_NOALLOC_SCRATCH_BYTES of sph.h


def sph_step_batched_noalloc(plan, store, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_step_batched_noalloc(_h(plan), _s(store), C.byref(p), C.byref(tuning) if tuning else None,
                                          _stream(stream)), "sph_step_batched_noalloc")


def sph_offload_bytes(layout: int, loop: int, n: int):
    a, b = sz(), sz()
    _check(lib().sph_offload_bytes(layout, loop, n, C.byref(a), C.byref(b)), "sph_offload_bytes")
    return a.value, b.value


def sph_offload_step(plan, host_store, dev_store, ws, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_offload_step(_h(plan), _s(host_store), _s(dev_store), C.byref(p),
                                  C.byref(tuning) if tuning else None, _ptr(ws), _nbytes(ws), _stream(stream)),
           "sph_offload_step")


def sph_offload_step_async(plan, host_store, dev_store, ws, nbundle=8, params=None, tuning=None, stream=None):
    p = params if params is not None else default_params()
    _check(lib().sph_offload_step_async(_h(plan), _s(host_store), _s(dev_store), C.byref(p),
                                        C.byref(tuning) if tuning else None, int(nbundle), _ptr(ws), _nbytes(ws),
                                        _stream(stream)),
           "sph_offload_step_async")


class Graph:
    """An executable HIP graph of one batched step."""

    def __init__(self, plan, store, ws, params=None, tuning=None):
        p = params if params is not None else default_params()
        out = vp()
        _check(lib().sph_graph_capture(_h(plan), _s(store), C.byref(p), C.byref(tuning) if tuning else None,
                                       _ptr(ws), _nbytes(ws), C.byref(out)), "sph_graph_capture")
        self.ptr = out.value
        self._keep = (plan, store, ws)

    def launch(self, stream=None):
        _check(lib().sph_graph_launch(self.ptr, _stream(stream)), "sph_graph_launch")

    def close(self):
        if self.ptr:
            lib().sph_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# convenience
# ---------------------------------------------------------------------------
def alloc_range_buffers(plan: Plan, loop: int, t0: int, t1: int, device="cuda"):
    import torch
    ns, pb, rb = plan.buffer_bytes(loop, t0, t1)
    pack = torch.empty(max(pb, 256), dtype=torch.uint8, device=device)
    res = torch.empty(max(rb, 256), dtype=torch.uint8, device=device)
    return ns, pack, res


def interact_ws(plan: Plan, loop: int = 2, device="cuda"):
    """Workspace of sph_interact_cells (the force loop's covers every loop)."""
    import torch
    return torch.zeros(sph_interact_ws_bytes(plan, loop), dtype=torch.uint8, device=device)


def cell_buffers(plan: Plan, loop: int, device="cuda"):
    """Pack / result buffers of the batched form (P = n rounded up to 64)."""
    import torch
    info = plan.info()
    P = (plan.n + 63) // 64 * 64
    pf, rp = sph_pack_layout(loop)
    pack = torch.empty(P * 4 * sum(pf) + info.ntile * 32 + 256, dtype=torch.uint8, device=device)
    res = torch.empty(P * 4 * rp + 256, dtype=torch.uint8, device=device)
    return pack, res
