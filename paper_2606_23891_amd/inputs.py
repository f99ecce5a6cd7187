"""Seeded synthetic particle sets and their cell/task lists.

This module only *creates inputs*: particle positions and attributes, the
store order, the cells (octree leaves or a uniform grid) and the self/pair
task list that the paper's offload engine walks (Sec. 2.2 and 2.3).  It holds
none of the method's arithmetic: no kernel sums, no packing, no reductions.
Both the HIP path and the CPU oracle receive exactly what this module builds.

Workload recipes (all in the periodic unit cube, numpy PCG64 seeds):

* jittered cubic lattice: particles at (i + 1/2) d plus U(-0.1 d, 0.1 d) per
  coordinate, equal masses 1/N, smoothing length h = 1.2348 d;
* Gresho-Chan vortex (Sec. 3.4 uses a 256^3 glass-like Gresho set): azimuthal
  velocity 5R / 2-5R / 0 in the x-y plane about (1/2, 1/2), pressure from
  radial balance, u = P / ((gamma-1) rho0);
* clustered gas (stand-in for the EAGLE-derived set of Sec. 3.4): 30 % uniform
  background, 70 % in Plummer clumps with log-normal shares, h from the 48th
  neighbour distance, clamped to a 100x span.

Store order is a global Morton order of the positions, so every dyadic cell
(uniform grid or octree leaf) is one contiguous range and consecutive 64-particle
tiles inside a cell are spatially compact.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Optional

import numpy as np

#: Support radius over smoothing length for the cubic spline in the SWIFT
#: convention (H = gamma_k h); used here only to turn a neighbour distance into
#: an input h and to decide which octree leaves share a pair task.
SUPPORT_PER_H = float(np.sqrt(10.0 / 3.0))
#: Resolution parameter: h = ETA * lattice spacing (about 48 neighbours).
ETA = 1.2348
GAMMA_AD = 5.0 / 3.0

CELL_DTYPE = np.dtype([("loc", "<f8", (3,)), ("width", "<f8"), ("first", "<i8"),
                       ("count", "<i4"), ("pad", "<i4")])
TASK_DTYPE = np.dtype([("ci", "<i4"), ("cj", "<i4"), ("pad", "<i4", (2,)),
                       ("shift", "<f8", (3,))])
assert CELL_DTYPE.itemsize == 48 and TASK_DTYPE.itemsize == 40

#: Every logical particle field: (numpy dtype, components).  The cold block
#: stands for the attributes no interaction loop touches (Table 1's ellipsis).
FIELDS = {
    "x": ("<f8", 3), "v": ("<f4", 3), "a": ("<f4", 3), "mass": ("<f4", 1),
    "h": ("<f4", 1), "u": ("<f4", 1), "u_dt": ("<f4", 1), "rho": ("<f4", 1),
    "rho_dh": ("<f4", 1), "wcount": ("<f4", 1), "div_v": ("<f4", 1),
    "rot_v": ("<f4", 3), "lap_u": ("<f4", 1), "v_sig": ("<f4", 1),
    "alpha_v": ("<f4", 1), "alpha_d": ("<f4", 1), "time_bin": ("<i1", 1),
    "id": ("<i8", 1), "cold": ("<u8", 5),
}


@dataclasses.dataclass
class ParticleSet:
    """Particles in store order plus the cells and tasks over them."""
    fields: Dict[str, np.ndarray]
    cells: np.ndarray
    tasks: np.ndarray
    meta: dict

    @property
    def n(self) -> int:
        return int(self.fields["x"].shape[0])


# --------------------------------------------------------------------------
# Morton ordering
# --------------------------------------------------------------------------
MORTON_BITS = 21


def _spread3(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_keys(x: np.ndarray) -> np.ndarray:
    """63-bit Morton keys of positions in [0, 1)^3 (21 bits per axis)."""
    q = np.floor(np.mod(x, 1.0) * float(1 << MORTON_BITS)).astype(np.int64)
    q = np.clip(q, 0, (1 << MORTON_BITS) - 1)
    return (_spread3(q[:, 0]) << np.uint64(2)) | (_spread3(q[:, 1]) << np.uint64(1)) | _spread3(q[:, 2])


def _reorder(fields: Dict[str, np.ndarray], perm: np.ndarray) -> Dict[str, np.ndarray]:
    return {k: np.ascontiguousarray(v[perm]) for k, v in fields.items()}


# --------------------------------------------------------------------------
# particle sets
# --------------------------------------------------------------------------
def lattice_positions(n_side: int, rng: np.random.Generator, jitter: float = 0.1) -> np.ndarray:
    d = 1.0 / n_side
    i = np.arange(n_side, dtype=np.float64)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), -1).reshape(-1, 3)
    x = (g + 0.5) * d
    if jitter:
        x = x + rng.uniform(-jitter * d, jitter * d, size=x.shape)
    return x


def gresho_profile(x: np.ndarray, p_centre: float = 5.0):
    """Azimuthal velocity and internal energy of the Gresho-Chan vortex."""
    dx = x[:, 0] - 0.5
    dy = x[:, 1] - 0.5
    r = np.hypot(dx, dy)
    vphi = np.where(r < 0.2, 5.0 * r, np.where(r < 0.4, 2.0 - 5.0 * r, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        p_mid = p_centre + 12.5 * r * r + 4.0 - 20.0 * r + 4.0 * np.log(np.maximum(5.0 * r, 1e-300))
    p = np.where(r < 0.2, p_centre + 12.5 * r * r,
                 np.where(r < 0.4, p_mid, p_centre - 2.0 + 4.0 * np.log(2.0)))
    safe_r = np.where(r > 0, r, 1.0)
    v = np.zeros_like(x)
    v[:, 0] = np.where(r > 0, -vphi * dy / safe_r, 0.0)
    v[:, 1] = np.where(r > 0, vphi * dx / safe_r, 0.0)
    u = p / ((GAMMA_AD - 1.0) * 1.0)
    return v, u


def _base_fields(x, v, u, m, h, alpha_v, alpha_d) -> Dict[str, np.ndarray]:
    n = x.shape[0]
    return {
        "x": np.ascontiguousarray(x, dtype=np.float64),
        "v": np.ascontiguousarray(v, dtype=np.float32),
        "mass": np.full(n, m, dtype=np.float32) if np.isscalar(m) else np.asarray(m, np.float32),
        "h": np.full(n, h, dtype=np.float32) if np.isscalar(h) else np.asarray(h, np.float32),
        "u": np.ascontiguousarray(u, dtype=np.float32),
        "alpha_v": np.asarray(alpha_v, dtype=np.float32),
        "alpha_d": np.asarray(alpha_d, dtype=np.float32),
    }


def lattice_set(n_side: int, seed: int, jitter: float = 0.1, velocity: str = "zero",
                u0: float = 1.0, switches: bool = False, v_disp: float = 0.0) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    x = lattice_positions(n_side, rng, jitter)
    n = x.shape[0]
    if velocity == "gresho":
        v, u = gresho_profile(x)
    else:
        v = np.zeros_like(x)
        u = np.full(n, u0)
    if v_disp:
        v = v + rng.normal(0.0, v_disp, v.shape)
    if switches:
        av = rng.uniform(0.1, 2.0, n)
        ad = rng.uniform(0.0, 1.0, n)
    else:
        av = np.ones(n)
        ad = np.zeros(n)
    return _base_fields(x, v, u, 1.0 / n, ETA / n_side, av, ad)


def clustered_set(n_side: int = 188, seed: int = 4, n_clumps: int = 256, a0: float = 0.0015,
                  bg_frac: float = 0.3, h_span: float = 100.0, workers: int = -1) -> Dict[str, np.ndarray]:
    """Uniform background plus Plummer clumps; h from the 48th neighbour."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    n = n_side ** 3
    n_bg = int(round(bg_frac * n))
    n_cl = n - n_bg
    shares = rng.lognormal(0.0, 1.0, n_clumps)
    counts = rng.multinomial(n_cl, shares / shares.sum())
    centres = rng.uniform(0.0, 1.0, (n_clumps, 3))
    med = float(np.median(counts[counts > 0]))
    a = a0 * np.cbrt(np.maximum(counts, 1) / med)
    # Plummer radius by inverse CDF, truncated at 10 a (U capped where r = 10 a).
    u_max = (1.0 + 0.01) ** -1.5
    cid = np.repeat(np.arange(n_clumps), counts)
    uu = rng.uniform(0.0, u_max, n_cl)
    rad = a[cid] / np.sqrt(uu ** (-2.0 / 3.0) - 1.0)
    dirn = rng.normal(size=(n_cl, 3))
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    x = np.empty((n, 3))
    x[:n_bg] = rng.uniform(0.0, 1.0, (n_bg, 3))
    x[n_bg:] = np.mod(centres[cid] + rad[:, None] * dirn, 1.0)
    bulk = rng.normal(0.0, 0.1, (n_clumps, 3))
    v = rng.normal(0.0, 0.05, (n, 3))
    v[n_bg:] += bulk[cid]
    tree = cKDTree(x, boxsize=1.0)
    dist, _ = tree.query(x, k=50, workers=workers)
    # support radius midway between the 48th and 49th neighbour (index 0 is
    # the particle itself), so no neighbour sits on the support edge
    r48 = 0.5 * (dist[:, 48] + dist[:, 49])
    h = r48 / SUPPORT_PER_H
    h = np.maximum(h, h.max() / h_span)
    m = 1.0 / n
    rho_hat = 49.0 * m / (4.0 / 3.0 * np.pi * (SUPPORT_PER_H * h) ** 3)
    u = 1.0 * rho_hat ** (2.0 / 3.0)
    av = rng.uniform(0.1, 2.0, n)
    ad = rng.uniform(0.0, 1.0, n)
    return _base_fields(x, v, u, m, h, av, ad)


# --------------------------------------------------------------------------
# cells and tasks
# --------------------------------------------------------------------------
def _sort_morton(fields):
    keys = morton_keys(fields["x"])
    perm = np.argsort(keys, kind="stable")
    return _reorder(fields, perm), keys[perm]


def uniform_grid(fields: Dict[str, np.ndarray], nc: int):
    """Morton-sort particles and build an nc^3 grid with self + 13 forward pair tasks per cell."""
    assert nc >= 3 and (nc & (nc - 1)) == 0, "grid side must be a power of two >= 4"
    fields, keys = _sort_morton(fields)
    lvl = int(np.log2(nc))
    ckey = keys >> np.uint64(3 * (MORTON_BITS - lvl))
    ncell = nc ** 3
    counts = np.bincount(ckey.astype(np.int64), minlength=ncell)
    first = np.concatenate([[0], np.cumsum(counts)[:-1]])
    # cell k (Morton index) -> integer coordinates
    kk = np.arange(ncell, dtype=np.uint64)
    coords = np.zeros((ncell, 3), dtype=np.int64)
    for b in range(lvl):
        for d in range(3):
            bit = (kk >> np.uint64(3 * b + (2 - d))) & np.uint64(1)
            coords[:, d] |= (bit.astype(np.int64) << b)
    w = 1.0 / nc
    cells = np.zeros(ncell, CELL_DTYPE)
    cells["loc"] = coords * w
    cells["width"] = w
    cells["first"] = first
    cells["count"] = counts
    lin = (coords[:, 0] * nc + coords[:, 1]) * nc + coords[:, 2]
    lin2morton = np.empty(ncell, np.int64)
    lin2morton[lin] = np.arange(ncell)
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
            if (a, b, c) > (0, 0, 0)]
    assert len(offs) == 13
    tasks = np.zeros(ncell * 14, TASK_DTYPE)
    idx = np.arange(ncell)
    # task order: for every cell in Morton order, its self task then its 13 forward pairs
    tasks["ci"] = np.repeat(idx, 14)
    cj = np.empty((ncell, 14), np.int64)
    shift = np.zeros((ncell, 14, 3))
    cj[:, 0] = idx
    for t, o in enumerate(offs, start=1):
        nb = coords + np.array(o)
        wrapped = np.mod(nb, nc)
        shift[:, t, :] = (nb - wrapped) // nc
        cj[:, t] = lin2morton[(wrapped[:, 0] * nc + wrapped[:, 1]) * nc + wrapped[:, 2]]
    tasks["cj"] = cj.reshape(-1)
    tasks["shift"] = shift.reshape(-1, 3).astype(np.float64)
    return fields, cells, tasks


def octree(fields: Dict[str, np.ndarray], top: int = 32, max_count: int = 2000, min_count: int = 10):
    """Octree leaves under a top-level top^3 grid (cells at least as wide as
    the largest support), split while they hold more than max_count particles
    -- also below the largest support radius in the leaf, as SWIFT's cells of a
    clustered set are.  A leaf with fewer than min_count particles is merged
    with the leaf next to it in store order (the smaller of the two, within
    the same top-level cell and while the sum stays within max_count); the
    merged cell is the smallest octree cube holding both, so it may overlap
    other cells, which the pair criterion below handles like any other gap 0.
    Pair tasks join every two cells whose boxes are closer than the larger of
    their largest support radii (Sec. 2.2: every neighbour of a particle then
    lies in a cell that shares a task with its own)."""
    fields, keys = _sort_morton(fields)
    hsup = SUPPORT_PER_H * fields["h"].astype(np.float64)
    assert hsup.max() < 1.0 / top, "top-level cells must be wider than the largest support"
    ltop = int(np.log2(top))
    leaves = []  # [level, key prefix, first, count]
    stack = []
    tkey = (keys >> np.uint64(3 * (MORTON_BITS - ltop))).astype(np.int64)
    tcounts = np.bincount(tkey, minlength=top ** 3)
    tfirst = np.concatenate([[0], np.cumsum(tcounts)[:-1]])
    for k in range(top ** 3):
        if tcounts[k]:
            stack.append((ltop, k, int(tfirst[k]), int(tcounts[k])))
    while stack:
        lvl, pre, f, c = stack.pop()
        if c > max_count and lvl < MORTON_BITS:
            sub = (keys[f:f + c] >> np.uint64(3 * (MORTON_BITS - lvl - 1))).astype(np.int64)
            for ch in range(7, -1, -1):
                cpre = (pre << 3) | ch
                lo = int(np.searchsorted(sub, cpre, "left"))
                hi = int(np.searchsorted(sub, cpre, "right"))
                if hi > lo:
                    stack.append((lvl + 1, cpre, f + lo, hi - lo))
        else:
            leaves.append([lvl, pre, f, c])
    leaves.sort(key=lambda t: t[2])

    def common(a, b):
        """the smallest octree cube (level, prefix) holding cubes a and b"""
        la, pa, lb, pb = a[0], a[1], b[0], b[1]
        lvl = min(la, lb)
        pa >>= 3 * (la - lvl)
        pb >>= 3 * (lb - lvl)
        while pa != pb:
            pa >>= 3
            pb >>= 3
            lvl -= 1
        return lvl, pa

    merged = True
    while merged:
        merged = False
        k = 0
        while k < len(leaves):
            if leaves[k][3] >= min_count:
                k += 1
                continue
            best = None
            for nb in (k - 1, k + 1):
                if 0 <= nb < len(leaves) and leaves[nb][3] + leaves[k][3] <= max_count:
                    lvl, pre = common(leaves[k], leaves[nb])
                    if lvl >= ltop and (best is None or leaves[nb][3] < leaves[best][3]):
                        best = nb
            if best is None:
                k += 1
                continue
            a_, b_ = sorted((k, best))
            lvl, pre = common(leaves[a_], leaves[b_])
            leaves[a_] = [lvl, pre, leaves[a_][2], leaves[a_][3] + leaves[b_][3]]
            del leaves[b_]
            merged = True
            k = a_
    leaves = [(l[0], l[1], l[2], l[3], float(hsup[l[2]:l[2] + l[3]].max())) for l in leaves]
    nl = len(leaves)
    lvl = np.array([t[0] for t in leaves])
    pre = np.array([t[1] for t in leaves], dtype=np.int64)
    cells = np.zeros(nl, CELL_DTYPE)
    cells["first"] = [t[2] for t in leaves]
    cells["count"] = [t[3] for t in leaves]
    hmax = np.array([t[4] for t in leaves])
    # decode cube corners
    coords = np.zeros((nl, 3), dtype=np.int64)
    for b in range(MORTON_BITS):
        for d in range(3):
            bit = (pre >> (3 * b + (2 - d))) & 1
            coords[:, d] |= bit << b
    cells["width"] = 1.0 / (1 << lvl)
    cells["loc"] = coords * cells["width"][:, None]
    # candidate pairs via the top-level grid
    ltop_of = (pre >> (3 * (lvl - ltop))).astype(np.int64)
    order = np.argsort(ltop_of, kind="stable")
    tstart = np.searchsorted(ltop_of[order], np.arange(top ** 3), "left")
    tend = np.searchsorted(ltop_of[order], np.arange(top ** 3), "right")
    tc = np.zeros((top ** 3, 3), np.int64)
    kk = np.arange(top ** 3, dtype=np.int64)
    for b in range(ltop):
        for d in range(3):
            tc[:, d] |= ((kk >> (3 * b + (2 - d))) & 1) << b
    lin2m = np.empty(top ** 3, np.int64)
    lin2m[(tc[:, 0] * top + tc[:, 1]) * top + tc[:, 2]] = kk
    centre = cells["loc"] + 0.5 * cells["width"][:, None]
    pa, pb = [], []
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    leaf_t = ltop_of
    for o in offs:
        nbt = np.mod(tc[leaf_t] + np.array(o), top)
        nbk = lin2m[(nbt[:, 0] * top + nbt[:, 1]) * top + nbt[:, 2]]
        s, e = tstart[nbk], tend[nbk]
        cnt = e - s
        a_idx = np.repeat(np.arange(nl), cnt)
        pos = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
        b_idx = order[np.repeat(s, cnt) + pos]
        keep = a_idx < b_idx
        pa.append(a_idx[keep])
        pb.append(b_idx[keep])
    pa = np.concatenate(pa)
    pb = np.concatenate(pb)
    pair = np.unique(pa * nl + pb)
    pa, pb = pair // nl, pair % nl
    d = centre[pb] - centre[pa]
    shift = -np.round(d)
    gap = np.maximum(0.0, np.abs(d + shift) - 0.5 * (cells["width"][pa] + cells["width"][pb])[:, None])
    dist = np.sqrt((gap ** 2).sum(1))
    keep = dist < np.maximum(hmax[pa], hmax[pb])
    pa, pb, shift = pa[keep], pb[keep], shift[keep]
    ntask = nl + pa.size
    tasks = np.zeros(ntask, TASK_DTYPE)
    # order: self task of each leaf, then its pair tasks (as ci)
    ci_all = np.concatenate([np.arange(nl), pa])
    cj_all = np.concatenate([np.arange(nl), pb])
    sh_all = np.concatenate([np.zeros((nl, 3)), shift])
    kind = np.concatenate([np.zeros(nl), np.ones(pa.size)])
    o2 = np.lexsort((cj_all, kind, ci_all))
    tasks["ci"] = ci_all[o2]
    tasks["cj"] = cj_all[o2]
    tasks["shift"] = sh_all[o2]
    return fields, cells, tasks


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def make_config(k: int, *, jitter: float = 0.1, grid: Optional[int] = None,
                n_side: Optional[int] = None) -> ParticleSet:
    """Build workload k (0..4) with seed k+1.

    0: 16^3 jittered lattice, zero velocity, u = 1, 4^3 cells.
    1: 64^3 Gresho vortex, 16^3 cells, random switches.
    2: 256^3 Gresho vortex, 32^3 cells (grid=64 gives the 64-per-cell variant).
    3: 188^3 clustered set on an octree (10..2000 particles per cell).
    4: 32^3 Gresho vortex on a jittered lattice, 8^3 cells (adjoint workload).
    ``n_side`` shrinks a workload for quick tests.
    """
    seed = k + 1
    if k == 0:
        ns = n_side or 16
        f = lattice_set(ns, seed, jitter)
        nc = grid or max(4, ns // 4)
    elif k in (1, 2, 4):
        ns = n_side or {1: 64, 2: 256, 4: 32}[k]
        # the adjoint workload adds a small velocity dispersion: where v = 0 exactly
        # (outside the vortex) pairs sit on the viscosity switch-on v_ij . r = 0,
        # at which L = sum |a|^2 has no derivative
        f = lattice_set(ns, seed, jitter, velocity="gresho", switches=True, v_disp=0.02 if k == 4 else 0.0)
        nc = grid or max(4, ns // {1: 4, 2: 8, 4: 4}[k])
    elif k == 3:
        ns = n_side or 188
        f = clustered_set(ns, seed)
        hsup = SUPPORT_PER_H * float(f["h"].max())
        top = 32
        while top > 1 and hsup >= 1.0 / top:
            top //= 2
        f, cells, tasks = octree(f, top=top)
        return ParticleSet(f, cells, tasks, {"config": k, "n_side": ns})
    else:
        raise ValueError(k)
    f, cells, tasks = uniform_grid(f, nc)
    return ParticleSet(f, cells, tasks, {"config": k, "n_side": ns, "grid": nc})


def random_fields(n: int, seed: int, x: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Random finite values for every field (for byte-exact pack/unpack tests)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, (dt, nc) in FIELDS.items():
        shape = (n, nc) if nc > 1 else (n,)
        if name == "x":
            out[name] = rng.uniform(0.0, 1.0, shape) if x is None else np.array(x, np.float64)
        elif dt == "<f4":
            out[name] = rng.uniform(-2.0, 2.0, shape).astype(np.float32)
        elif dt == "<i1":
            out[name] = rng.integers(-128, 128, shape, dtype=np.int8)
        elif dt == "<i8":
            out[name] = rng.integers(-2 ** 62, 2 ** 62, shape, dtype=np.int64)
        else:
            out[name] = rng.integers(0, 2 ** 63, shape, dtype=np.uint64)
    return out


def cell_stats(cells: np.ndarray) -> dict:
    c = cells["count"]
    return {"ncell": int(c.size), "min": int(c.min()), "max": int(c.max()),
            "mean": float(c.mean()), "median": float(np.median(c))}
