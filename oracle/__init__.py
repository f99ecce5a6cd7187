"""CPU oracle for the SPH pack / interact / unpack path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke entry and the benchmark's CPU
baseline leg are the only callers.  The product package never imports it.

Wraps ``sph_oracle.c`` (plain C, FP64, OpenMP brute force) through ctypes.
``build()`` compiles it with gcc; ``lib()`` loads it (building when missing).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sph_oracle.c")
SO = os.path.join(HERE, "liboracle.so")

LOOPS = {"density": 0, "gradient": 1, "force": 2}
LAYOUTS = ["AOS", "AOS_RANDOM", "SAOS_GRAD", "SAOS_FORCE", "SAOS_SHARED", "SAOS_GRAD_TYPE",
           "SAOS_FORCE_TYPE", "SAOS_SHARED_TYPE", "SOA", "SAOS_SHARED_REPL"]
FIELD_IDS = {"x": 0, "v": 1, "a": 2, "mass": 3, "h": 4, "u": 5, "u_dt": 6, "rho": 7, "rho_dh": 8,
             "wcount": 9, "div_v": 10, "rot_v": 11, "lap_u": 12, "v_sig": 13, "alpha_v": 14,
             "alpha_d": 15, "time_bin": 16, "id": 17, "cold": 18}
PACK_PLANES = {0: (4, 1), 1: (4, 4, 2), 2: (4, 4, 4, 4, 1)}   # floats per plane
RESULT_PLANES = {0: 3, 1: 6, 2: 4}
#: dense host representation of each field: (numpy dtype, components)
FIELD_TYPES = {"x": ("<f8", 3), "v": ("<f4", 3), "a": ("<f4", 3), "mass": ("<f4", 1),
               "h": ("<f4", 1), "u": ("<f4", 1), "u_dt": ("<f4", 1), "rho": ("<f4", 1),
               "rho_dh": ("<f4", 1), "wcount": ("<f4", 1), "div_v": ("<f4", 1),
               "rot_v": ("<f4", 3), "lap_u": ("<f4", 1), "v_sig": ("<f4", 1),
               "alpha_v": ("<f4", 1), "alpha_d": ("<f4", 1), "time_bin": ("<i1", 1),
               "id": ("<i8", 1), "cold": ("<u8", 5)}

_lib = None


def build(force: bool = True) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
           "-std=c11", "-Wall", "-o", SO, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return SO


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        build()
    L = C.CDLL(SO)
    d, i32, i64, vp, sz = C.c_double, C.c_int32, C.c_int64, C.c_void_p, C.c_size_t
    for name in ("or_w", "or_dw", "or_gamma_k"):
        getattr(L, name).restype = d
    L.or_w.argtypes = [d]
    L.or_dw.argtypes = [d]
    for name in ("or_W", "or_dWdh", "or_F", "or_dWdr", "or_d2Wdhdr", "or_dFdr"):
        getattr(L, name).restype = d
        getattr(L, name).argtypes = [d, d]
    L.or_density.argtypes = [i64, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.or_gradient.argtypes = [i64, vp, vp, vp, vp, vp, vp, d, d, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                              vp]
    L.or_force.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, d, d, d, i64, vp, vp,
                           vp, vp, vp, vp, vp, vp, vp]
    L.or_cell_reach.argtypes = [i32, vp, vp, vp, i32, vp, vp, vp]
    L.or_grid_build.argtypes = [i64, vp, d]
    L.or_grid_build.restype = vp
    L.or_grid_free.argtypes = [vp]
    L.or_balsara.argtypes = [i64, vp, vp, vp, vp, vp, vp, d, d, vp]
    L.or_layout_info.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(sz)]
    L.or_x_copies.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(sz)]
    L.or_field_location.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(sz),
                                    C.POINTER(sz)]
    L.or_store_put.argtypes = [C.c_int, i64, vp, C.c_int, vp]
    L.or_store_get.argtypes = [C.c_int, i64, vp, C.c_int, vp]
    L.or_pack.argtypes = [C.c_int, C.c_int, i64, vp, vp, vp, i32, i32, vp]
    L.or_pack_cells.argtypes = [C.c_int, C.c_int, i64, vp, vp, i32, vp]
    L.or_unpack.argtypes = [C.c_int, C.c_int, i64, vp, vp, vp, i32, i32, vp]
    L.or_unpack_cells.argtypes = [C.c_int, C.c_int, i64, vp, vp]
    L.or_zero_outputs.argtypes = [C.c_int, C.c_int, i64, vp]
    L.or_range_slots.argtypes = [vp, vp, i32, i32]
    L.or_range_slots.restype = i64
    _lib = L
    return L


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------
# interaction loops
# --------------------------------------------------------------------------
GAMMA_AD = 5.0 / 3.0
BETA_VISC = 3.0
BALSARA_EPS = 1e-4


def _eps(epsx):
    return None if epsx is None else _c(epsx, np.float64)


class _Grid:
    """Candidate grid for a loop call (grid=True): cells at least as wide as
    the largest support (with the edge band's margin), so the loops skip only
    particles that cannot interact; None when the box holds fewer than 3
    cells per side (the loops then visit every particle)."""

    def __init__(self, use: bool, x: np.ndarray, h: np.ndarray, epsx):
        self.ptr = None
        if use and x.shape[0]:
            reach = 1.0001 * GAMMA_K * float(np.max(h)) + (0.0 if epsx is None else 2.0 * float(np.max(epsx)))
            self.ptr = lib().or_grid_build(x.shape[0], _p(x), reach)

    def __enter__(self):
        return self.ptr

    def __exit__(self, *exc):
        if self.ptr:
            lib().or_grid_free(self.ptr)


def density(x, m, h, rows=None, epsx=None, grid=False) -> Dict[str, np.ndarray]:
    """FP64 density sums.  S: arithmetic error scale; P: position error scale for
    the per-particle position resolution epsx (0 when epsx is None); band: pairs
    whose distance to the support edge is within 1e-6 H + epsx_i + epsx_j.
    grid=True visits candidates from a uniform grid instead of every particle
    (same results, bit for bit)."""
    L = lib()
    x = _c(x, np.float64); m = _c(m, np.float32); h = _c(h, np.float32)
    n = x.shape[0]
    rows = None if rows is None else _c(rows, np.int64)
    nr = n if rows is None else rows.size
    out = {k: np.zeros(nr) for k in ("rho", "rho_dh", "wcount")}
    S = np.zeros((nr, 3)); P = np.zeros((nr, 3)); cnt = np.zeros(nr, np.int32); band = np.zeros(nr, np.int32)
    epsx = _eps(epsx)
    with _Grid(grid, x, h, epsx) as g:
        L.or_density(n, _p(x), _p(m), _p(h), nr, _p(rows), _p(epsx), _p(out["rho"]), _p(out["rho_dh"]),
                     _p(out["wcount"]), _p(S), _p(P), _p(cnt), _p(band), g)
    out.update(S=S, P=P, count=cnt, band=band)
    return out


def gradient(x, v, m, h, u, rho, rows=None, gamma=GAMMA_AD, beta=BETA_VISC, epsx=None,
             grid=False) -> Dict[str, np.ndarray]:
    L = lib()
    x = _c(x, np.float64); v = _c(v, np.float32); m = _c(m, np.float32); h = _c(h, np.float32)
    u = _c(u, np.float32); rho = _c(rho, np.float64)
    n = x.shape[0]
    rows = None if rows is None else _c(rows, np.int64)
    nr = n if rows is None else rows.size
    D = np.zeros(nr); R = np.zeros((nr, 3)); Lp = np.zeros(nr); V = np.zeros(nr)
    S = np.zeros((nr, 5)); P = np.zeros((nr, 5)); cnt = np.zeros(nr, np.int32); band = np.zeros(nr, np.int32)
    epsx = _eps(epsx)
    with _Grid(grid, x, h, epsx) as g:
        L.or_gradient(n, _p(x), _p(v), _p(m), _p(h), _p(u), _p(rho), gamma, beta, nr, _p(rows), _p(epsx),
                      _p(D), _p(R), _p(Lp), _p(V), _p(S), _p(P), _p(cnt), _p(band), g)
    return {"div_v": D, "rot_v": R, "lap_u": Lp, "v_sig": V, "S": S, "P": P, "count": cnt, "band": band}


def force(x, v, m, h, u, rho, rho_dh, D, R, alpha_v, alpha_d, atilde=None, rows=None,
          gamma=GAMMA_AD, beta=BETA_VISC, eps=BALSARA_EPS, epsx=None, grid=False) -> Dict[str, np.ndarray]:
    L = lib()
    x = _c(x, np.float64); v = _c(v, np.float32); m = _c(m, np.float32); h = _c(h, np.float32)
    u = _c(u, np.float32); rho = _c(rho, np.float64); rho_dh = _c(rho_dh, np.float64)
    D = _c(D, np.float64); R = _c(R, np.float64)
    alpha_v = _c(alpha_v, np.float32); alpha_d = _c(alpha_d, np.float32)
    atilde = None if atilde is None else _c(atilde, np.float64)
    n = x.shape[0]
    rows = None if rows is None else _c(rows, np.int64)
    nr = n if rows is None else rows.size
    a = np.zeros((nr, 3)); udt = np.zeros(nr); S = np.zeros((nr, 4)); P = np.zeros((nr, 4))
    cnt = np.zeros(nr, np.int32); band = np.zeros(nr, np.int32)
    epsx = _eps(epsx)
    with _Grid(grid, x, h, epsx) as g:
        L.or_force(n, _p(x), _p(v), _p(m), _p(h), _p(u), _p(rho), _p(rho_dh), _p(D), _p(R),
                   _p(alpha_v), _p(alpha_d), _p(atilde), gamma, beta, eps, nr, _p(rows), _p(epsx),
                   _p(a), _p(udt), _p(S), _p(P), _p(cnt), _p(band), g)
    return {"a": a, "u_dt": udt, "S": S, "P": P, "count": cnt, "band": band}


def balsara(h, u, rho, D, R, alpha_v, gamma=GAMMA_AD, eps=BALSARA_EPS) -> np.ndarray:
    L = lib()
    h = _c(h, np.float32); u = _c(u, np.float32); rho = _c(rho, np.float64)
    D = _c(D, np.float64); R = _c(R, np.float64); alpha_v = _c(alpha_v, np.float32)
    out = np.zeros(h.size)
    L.or_balsara(h.size, _p(h), _p(u), _p(rho), _p(D), _p(R), _p(alpha_v), gamma, eps, _p(out))
    return out


GAMMA_K = np.sqrt(10.0 / 3.0)   # support H over smoothing length h (cubic spline)


def cell_reach(cells, tasks) -> np.ndarray:
    """Per cell, the smallest gap (minimum image) between its cube and the
    cube of a non-empty cell that shares no task with it, at most 1/2: the
    distance within which every neighbour of the cell's particles lies in a
    cell joined to it by a task (Sec. 2.2).  Brute force over cell pairs."""
    L = lib()
    nc, nt = len(cells), len(tasks)
    loc = _c(cells["loc"], np.float64); width = _c(cells["width"], np.float64)
    count = _c(cells["count"], np.int32)
    ci = _c(tasks["ci"], np.int32); cj = _c(tasks["cj"], np.int32)
    out = np.zeros(nc)
    L.or_cell_reach(nc, _p(loc), _p(width), _p(count), nt, _p(ci), _p(cj), _p(out))
    return out


def particle_reach(cells, tasks, n) -> np.ndarray:
    """the reach of every particle's cell (cells hold consecutive particle ranges)"""
    r = cell_reach(cells, tasks)
    out = np.zeros(n)
    for c in range(len(cells)):
        out[cells["first"][c]:cells["first"][c] + cells["count"][c]] = r[c]
    return out


def h_newton_step(h, m, rho, rho_dh, reach, eta, tol):
    """One smoothing-length update per particle, in FP64 (h itself is a float32
    field).  Root sought: f(h) = rho(h) h^3 - m eta^3 = 0, i.e. h = eta (m /
    rho)^(1/3).  Newton: dh = -f / f' with f' = h^3 rho' + 3 h^2 rho, which is
    dh = -h (rho - n) / (3 rho + h rho') for n = m eta^3 / h^3; where that
    denominator is not positive, the fixed-point step to eta (m / rho)^(1/3).
    |dh| <= tol h: converged, h kept; otherwise h + dh clipped to [h/2, 2h].
    Either way h is then held to gamma_K h <= the reach of the particle's cell
    (cell_reach: the support its cell's tasks cover; a particle above it
    moves even when converged).  Returns (new h as float32, moved mask)."""
    h64 = np.asarray(h, np.float64)
    rho = np.asarray(rho, np.float64)
    n = np.asarray(m, np.float64) * eta ** 3 / h64 ** 3
    den = 3.0 * rho + h64 * np.asarray(rho_dh, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        newton = -h64 * (rho - n) / den
    fixed = h64 * (np.cbrt(n / rho) - 1.0)
    dh = np.where(den > 0.0, newton, fixed)
    conv = np.abs(dh) <= tol * h64
    hn = np.where(conv, h64, np.clip(h64 + dh, 0.5 * h64, 2.0 * h64))
    hn = np.minimum(hn, np.asarray(reach, np.float64) / GAMMA_K)
    hn32 = hn.astype(np.float32)
    moved = hn32 != np.asarray(h, np.float32)
    out = np.asarray(h, np.float32).copy()
    out[moved] = hn32[moved]
    return out, moved


def h_iterate(x, m, h, reach, eta=1.2348, tol=1e-4, max_iter=30, rows=None,
              grid=False) -> Dict[str, np.ndarray]:
    """The smoothing-length iteration: the FP64 brute-force density of the
    particles whose h moved (all on the first pass), then one h_newton_step
    for them, until none moves or max_iter passes.  Returns the final h, the
    density outputs belonging to it, the passes run and the particles that
    still moved in the last pass.

    rows: iterate only these particles.  A particle's density depends on its
    own h alone, so each row ends exactly as in the iteration of the whole
    set; the other particles keep their h (and zero density outputs), and
    passes / unconverged count the rows only.  grid: the density's candidate
    grid mode (the same sums)."""
    h = np.asarray(h, np.float32).copy()
    n = h.size
    width = np.asarray(reach, np.float64)
    rho, rdh, wc = np.zeros(n), np.zeros(n), np.zeros(n)
    rows = np.arange(n) if rows is None else np.unique(np.asarray(rows, np.int64))
    passes, still = 0, 0
    for _ in range(max_iter):
        if rows.size == 0:
            break
        d = density(x, m, h, rows=rows, grid=grid)
        rho[rows], rdh[rows], wc[rows] = d["rho"], d["rho_dh"], d["wcount"]
        hn, moved = h_newton_step(h[rows], np.asarray(m)[rows], rho[rows], rdh[rows], width[rows], eta, tol)
        h[rows] = hn
        passes += 1
        still = int(moved.sum())
        rows = rows[moved]
        if still == 0:
            break
    return {"h": h, "rho": rho, "rho_dh": rdh, "wcount": wc, "passes": passes, "unconverged": still}


# --------------------------------------------------------------------------
# time integration around the loops (kick-drift-kick leapfrog, one global dt)
# --------------------------------------------------------------------------
def kick(v, a, u, u_dt, dt):
    """v + a dt and u + u_dt dt in float32, the product rounded, then the sum"""
    f32 = np.float32
    dt = f32(dt)
    v = np.asarray(v, f32); a = np.asarray(a, f32); u = np.asarray(u, f32); u_dt = np.asarray(u_dt, f32)
    return (v + (a * dt).astype(f32)).astype(f32), (u + (u_dt * dt).astype(f32)).astype(f32)


def drift(x, v, dt, cells):
    """x + v dt in float64 (v widened exactly), and for every particle the
    Euclidean distance by which it lies outside its cell's cube afterwards"""
    x = np.asarray(x, np.float64)
    xn = x + np.asarray(v, np.float32).astype(np.float64) * float(dt)
    loc = np.repeat(np.asarray(cells["loc"], np.float64), np.asarray(cells["count"]), axis=0)
    w = np.repeat(np.asarray(cells["width"], np.float64), np.asarray(cells["count"]))[:, None]
    e = np.maximum(np.maximum(loc - xn, xn - (loc + w)), 0.0)
    return xn, np.sqrt((e * e).sum(1))


def cfl_dt(h, v_sig, cfl):
    """min over particles with V > 0 of (cfl (gamma_K h)) / V in float32 (+inf if none)"""
    f32 = np.float32
    h = np.asarray(h, f32); vs = np.asarray(v_sig, f32)
    gk = f32(lib().or_gamma_k())
    sel = vs > 0
    if not sel.any():
        return f32(np.inf)
    return ((f32(cfl) * (gk * h[sel]).astype(f32)).astype(f32) / vs[sel]).astype(f32).min()


def step_kdk(f: Dict[str, np.ndarray], cells, dt):
    """kick by dt/2 (the given a, u_dt), drift by dt, FP64 density -> gradient
    -> force at the new positions, kick by dt/2 with the new a, u_dt (rounded to
    the store's float32).  Returns the new fields and the three loops' results."""
    f = dict(f)
    half = np.float32(0.5) * np.float32(dt)
    f["v"], f["u"] = kick(f["v"], f["a"], f["u"], f["u_dt"], half)
    f["x"], _ = drift(f["x"], f["v"], np.float64(np.float32(dt)), cells)
    r = full_chain(f)
    a32 = r["force"]["a"].astype(np.float32)
    udt32 = r["force"]["u_dt"].astype(np.float32)
    f["v"], f["u"] = kick(f["v"], a32, f["u"], udt32, half)
    f["a"], f["u_dt"] = a32, udt32
    return f, r


def pack_resolution(cells) -> np.ndarray:
    """Per-particle position resolution of the packed FP32 offsets: 2^-22 times
    the width of the particle's cell (offsets span at most a few cell widths and
    are rounded once, plus once more when translated between cell frames)."""
    return np.repeat(np.asarray(cells["width"], np.float64), np.asarray(cells["count"])) * 2.0 ** -22


def full_chain(f: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """FP64 density -> gradient -> force on the logical fields of a particle set."""
    d = density(f["x"], f["mass"], f["h"])
    g = gradient(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"])
    fo = force(f["x"], f["v"], f["mass"], f["h"], f["u"], d["rho"], d["rho_dh"], g["div_v"],
               g["rot_v"], f["alpha_v"], f["alpha_d"])
    return {"density": d, "gradient": g, "force": fo}


# --------------------------------------------------------------------------
# layouts, store, pack / unpack
# --------------------------------------------------------------------------
def x_copies(layout: int):
    """[(substruct, byte offset of x[0])] of the copies of x after the one that is read"""
    L = lib()
    n = C.c_int()
    sb = (C.c_int * 4)()
    of = (C.c_size_t * 4)()
    if L.or_x_copies(layout, C.byref(n), sb, of):
        raise ValueError(layout)
    return [(sb[r], of[r]) for r in range(n.value)]


def layout_info(layout: int):
    L = lib()
    ns = C.c_int()
    sb = (C.c_size_t * 32)()
    if L.or_layout_info(layout, C.byref(ns), sb):
        raise ValueError(layout)
    return [int(sb[i]) for i in range(ns.value)]


def field_location(layout: int, field: int, comp: int):
    L = lib()
    s, o, st = C.c_int(), C.c_size_t(), C.c_size_t()
    if L.or_field_location(layout, field, comp, C.byref(s), C.byref(o), C.byref(st)):
        raise ValueError((layout, field, comp))
    return s.value, o.value, st.value


class HostStore:
    """A particle store in host memory, laid out by the oracle's own tables."""

    def __init__(self, layout: int, n: int, fill: int = 0):
        self.layout, self.n = layout, n
        self.sub_bytes = layout_info(layout)
        self.subs = [np.full(n * b, fill, np.uint8) for b in self.sub_bytes]
        self._ptrs = (C.c_void_p * 32)(*[s.ctypes.data for s in self.subs])

    @property
    def ptrs(self):
        return self._ptrs

    def put(self, name: str, arr: np.ndarray):
        dt, nc = FIELD_TYPES[name]
        a = np.ascontiguousarray(arr, dtype=dt)
        assert a.size == self.n * nc
        if lib().or_store_put(self.layout, self.n, self._ptrs, FIELD_IDS[name], a.ctypes.data):
            raise ValueError(name)

    def get(self, name: str) -> np.ndarray:
        dt, nc = FIELD_TYPES[name]
        a = np.zeros((self.n, nc) if nc > 1 else (self.n,), dt)
        if lib().or_store_get(self.layout, self.n, self._ptrs, FIELD_IDS[name], a.ctypes.data):
            raise ValueError(name)
        return a

    def put_all(self, fields: Dict[str, np.ndarray]):
        for k, v in fields.items():
            self.put(k, v)

    def raw(self) -> bytes:
        return b"".join(s.tobytes() for s in self.subs)


def round_slots(nslot: int) -> int:
    return (nslot + 63) // 64 * 64


def range_slots(cells, tasks, t0, t1) -> int:
    c = _c(cells, cells.dtype); t = _c(tasks, tasks.dtype)
    return int(lib().or_range_slots(c.ctypes.data, t.ctypes.data, t0, t1))


def pack_bytes(loop: int, nslot: int) -> int:
    return round_slots(nslot) * 4 * sum(PACK_PLANES[loop])


def result_bytes(loop: int, nslot: int) -> int:
    return round_slots(nslot) * 4 * RESULT_PLANES[loop]


def pack(store: HostStore, loop: int, cells, tasks, t0, t1) -> np.ndarray:
    c = _c(cells, cells.dtype); t = _c(tasks, tasks.dtype)
    ns = range_slots(c, t, t0, t1)
    buf = np.zeros(pack_bytes(loop, ns), np.uint8)
    if lib().or_pack(store.layout, loop, store.n, store.ptrs, c.ctypes.data, t.ctypes.data, t0, t1,
                     buf.ctypes.data):
        raise ValueError("pack")
    return buf


def pack_cells(store: HostStore, loop: int, cells) -> np.ndarray:
    c = _c(cells, cells.dtype)
    buf = np.zeros(pack_bytes(loop, store.n), np.uint8)
    if lib().or_pack_cells(store.layout, loop, store.n, store.ptrs, c.ctypes.data, c.size, buf.ctypes.data):
        raise ValueError("pack_cells")
    return buf


def unpack(store: HostStore, loop: int, cells, tasks, t0, t1, res: np.ndarray):
    c = _c(cells, cells.dtype); t = _c(tasks, tasks.dtype)
    r = np.ascontiguousarray(res)
    if lib().or_unpack(store.layout, loop, store.n, store.ptrs, c.ctypes.data, t.ctypes.data, t0, t1,
                       r.ctypes.data):
        raise ValueError("unpack")


def unpack_cells(store: HostStore, loop: int, res: np.ndarray):
    r = np.ascontiguousarray(res)
    if lib().or_unpack_cells(store.layout, loop, store.n, store.ptrs, r.ctypes.data):
        raise ValueError("unpack_cells")


def zero_outputs(store: HostStore, loop: int):
    if lib().or_zero_outputs(store.layout, loop, store.n, store.ptrs):
        raise ValueError("zero")
