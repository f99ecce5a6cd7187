"""The seeded input builders: cells tile the Morton-ordered store, every
particle lies in its cell, tasks reference valid cells with periodic shifts,
and the neighbour search through tasks is complete (checked by brute force)."""
import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs


def _check_cells_tasks(ps):
    c, t, x = ps.cells, ps.tasks, ps.fields["x"]
    assert c["first"][0] == 0 and np.all(c["first"][1:] == c["first"][:-1] + c["count"][:-1])
    assert c["first"][-1] + c["count"][-1] == ps.n
    for k in range(len(c)):
        xx = x[c["first"][k]:c["first"][k] + c["count"][k]]
        assert np.all(xx >= c["loc"][k]) and np.all(xx < c["loc"][k] + c["width"][k])
    assert np.all((t["ci"] >= 0) & (t["ci"] < len(c)) & (t["cj"] >= 0) & (t["cj"] < len(c)))
    self_ = t["ci"] == t["cj"]
    assert np.all(t["shift"][self_] == 0)
    assert self_.sum() == len(c)
    pairs = set(zip(t["ci"][~self_].tolist(), t["cj"][~self_].tolist()))
    assert len(pairs) == (~self_).sum()                        # each pair once
    assert not any((b, a) in pairs for a, b in pairs)          # and in one orientation


def _complete(ps, nsample=300, seed=0):
    """every neighbour (r < max(H_i, H_j)) of sampled particles is reachable
    through the particle's own cell's tasks"""
    c, t, x, h = ps.cells, ps.tasks, ps.fields["x"], ps.fields["h"].astype(float)
    H = inputs.SUPPORT_PER_H * h
    cell_of = np.repeat(np.arange(len(c)), c["count"])
    nb = {k: {k} for k in range(len(c))}
    for a, b in zip(t["ci"], t["cj"]):
        nb[a].add(b)
        nb[b].add(a)
    rows = np.random.default_rng(seed).choice(ps.n, min(nsample, ps.n), replace=False)
    for i in rows:
        d = x - x[i]
        d -= np.round(d)
        r = np.sqrt((d * d).sum(1))
        js = np.nonzero(r < np.maximum(H[i], H))[0]
        assert set(cell_of[js].tolist()) <= nb[cell_of[i]], i


@pytest.mark.parametrize("k,kw", [(0, {}), (0, {"n_side": 8, "grid": 4}), (4, {"n_side": 16}),
                                  (2, {"n_side": 32, "grid": 4}), (3, {"n_side": 24}), (3, {"n_side": 40})])
def test_small_workloads(k, kw):
    ps = inputs.make_config(k, **kw)
    _check_cells_tasks(ps)
    _complete(ps)


def test_lattice_stats_match_paper_shape():
    ps = inputs.make_config(1, n_side=32)
    st = inputs.cell_stats(ps.cells)
    assert st["min"] == st["max"] == 64   # 64 per cell like the Gresho256 run (Sec. 3.4)


def test_clustered_set_is_uneven():
    ps = inputs.make_config(3, n_side=40)
    st = inputs.cell_stats(ps.cells)
    h = ps.fields["h"]
    assert 10.0 < h.max() / h.min() <= 100.0 * (1 + 1e-6)       # span, clamped at 100
    assert st["max"] > 8 * st["median"]


def test_gresho_profile():
    x = np.array([[0.5 + r, 0.5, 0.3] for r in (0.0, 0.1, 0.2, 0.3, 0.4, 0.45)])
    v, u = inputs.gresho_profile(x)
    vphi = np.hypot(v[:, 0], v[:, 1])
    np.testing.assert_allclose(vphi, [0, 0.5, 1.0, 0.5, 0.0, 0.0], atol=1e-12)
    p = u * (2.0 / 3.0)
    # continuity at R = 0.2 and 0.4 and the outer value 3 + 4 ln 2
    np.testing.assert_allclose(p[2], 5.5, rtol=1e-12)
    np.testing.assert_allclose(p[4], 3.0 + 4.0 * np.log(2.0), rtol=1e-12)
    # radial balance dP/dR = v^2 / R by central differences
    for r0 in (0.1, 0.3):
        e = 1e-6
        xx = np.array([[0.5 + r0 - e, 0.5, 0.5], [0.5 + r0 + e, 0.5, 0.5], [0.5 + r0, 0.5, 0.5]])
        vv, uu = inputs.gresho_profile(xx)
        dp = (uu[1] - uu[0]) * (2.0 / 3.0) / (2 * e)
        np.testing.assert_allclose(dp, np.hypot(*vv[2, :2]) ** 2 / r0, rtol=1e-6)


def test_clustered_cells_within_counts():
    """the clustered workload's octree (at 64^3): every cell holds 10 to 2000
    particles, supports span close to the factor of 100 the full workload is
    clamped to, and cells narrower than their largest support exist (the
    octree splits on counts alone)"""
    ps = inputs.make_config(3, n_side=64)
    c = ps.cells["count"]
    assert c.min() >= 10 and c.max() <= 2000, inputs.cell_stats(ps.cells)
    h = ps.fields["h"]
    assert 50.0 <= float(h.max() / h.min()) <= 100.0 * (1 + 1e-6)
    H = inputs.SUPPORT_PER_H * h.astype(np.float64)
    hmax = np.maximum.reduceat(H, ps.cells["first"])
    assert np.any(hmax > ps.cells["width"])


def test_cell_reach_definition():
    """the oracle's cell reach: the cell width on a uniform grid with 26
    neighbour tasks; on the clustered octree, every particle within the reach
    of another's cell sits in a cell that shares a task with it (checked by
    brute force over sampled particles)"""
    ps = inputs.make_config(0)
    r = oracle.cell_reach(ps.cells, ps.tasks)
    np.testing.assert_array_equal(r, ps.cells["width"])
    ps = inputs.make_config(3, n_side=48)
    r = oracle.cell_reach(ps.cells, ps.tasks)
    x = ps.fields["x"]
    cell_of = np.repeat(np.arange(len(ps.cells)), ps.cells["count"])
    part = {(int(a), int(b)) for a, b in zip(ps.tasks["ci"], ps.tasks["cj"])}
    part |= {(b, a) for a, b in part}
    rng = np.random.default_rng(3)
    for i in rng.choice(ps.n, 400, replace=False):
        d = x - x[i]
        d -= np.round(d)
        near = np.flatnonzero(np.sqrt((d * d).sum(1)) < r[cell_of[i]])
        for j in near:
            ci, cj = int(cell_of[i]), int(cell_of[j])
            assert ci == cj or (ci, cj) in part, (i, j)
    assert np.any(r < 0.5)
