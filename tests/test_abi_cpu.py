"""C-ABI checks that need no GPU: exported symbols, the library's layout tables
against the oracle's independently written ones, and argument validation that
must fail before anything is enqueued."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2606_23891_amd import inputs, sph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "sph.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = sph.lib()
    names = declared_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(sph._SIGS), set(names) ^ set(sph._SIGS)


@pytest.mark.parametrize("layout", range(10))
def test_layout_tables_match_oracle(layout):
    assert sph.sph_layout_info(layout) == oracle.layout_info(layout)
    assert sph.sph_x_replicas(layout) == oracle.x_copies(layout)
    for name, fid in sph.FIELD_ID.items():
        nc, cb = sph.sph_field_info(fid)
        assert (nc, cb) == (oracle.FIELD_TYPES[name][1], np.dtype(oracle.FIELD_TYPES[name][0]).itemsize)
        for c in range(nc):
            assert sph.sph_field_location(layout, fid, c) == oracle.field_location(layout, fid, c)


def test_pack_record_matches_oracle():
    for loop in range(3):
        planes, rp = sph.sph_pack_layout(loop)
        assert tuple(planes) == oracle.PACK_PLANES[loop]
        assert rp == oracle.RESULT_PLANES[loop]


# members of the force record in plane order, the subsets density and
# gradient pack, and each loop's result planes (field, component)
_MEMBERS = [("x", 0), ("x", 1), ("x", 2), ("h", 0), ("v", 0), ("v", 1), ("v", 2), ("mass", 0), ("u", 0),
            ("rho", 0), ("rho_dh", 0), ("div_v", 0), ("rot_v", 0), ("rot_v", 1), ("rot_v", 2), ("alpha_v", 0),
            ("alpha_d", 0)]
_LOOP_MEMBERS = [[0, 1, 2, 3, 7], list(range(10)), list(range(17))]
_RESULTS = [[("rho", 0), ("rho_dh", 0), ("wcount", 0)],
            [("div_v", 0), ("rot_v", 0), ("rot_v", 1), ("rot_v", 2), ("lap_u", 0), ("v_sig", 0)],
            [("a", 0), ("a", 1), ("a", 2), ("u_dt", 0)]]


@pytest.mark.parametrize("layout", range(10))
def test_fission_passes_partition_by_schedule_key(layout):
    """every schedule's pass masks partition the loop's members, members of a
    pass share the schedule's key (none / substruct / field / component type /
    both) read from the layout tables, passes differ in it and come in the
    order of their first member"""
    for loop in range(3):
        packs = [(_MEMBERS[k], k) for k in _LOOP_MEMBERS[loop]]
        unpacks = [(fc, k) for k, fc in enumerate(_RESULTS[loop])]
        for sched in range(5):
            pm, um = sph.sph_fission_passes(layout, loop, sched)
            for masks, mem in ((pm, packs), (um, unpacks)):
                def key(fc):
                    fid = sph.FIELD_ID[fc[0]]
                    sub = sph.sph_field_location(layout, fid, fc[1])[0]
                    nbytes = sph.sph_field_info(fid)[1]
                    return [0, sub, fid, nbytes, (sub, nbytes)][sched]
                want_order, groups = [], {}
                for fc, bit in mem:
                    kk = key(fc)
                    if kk not in groups:
                        want_order.append(kk)
                        groups[kk] = 0
                    groups[kk] |= 1 << bit
                assert masks == [groups[kk] for kk in want_order], (layout, loop, sched)
                union = 0
                for m in masks:
                    assert m and not (union & m)
                    union |= m
                assert union == sum(1 << bit for _, bit in mem)
            if sched == 0:
                assert len(pm) == 1 and len(um) == 1
    with pytest.raises(sph.SphError):
        sph.sph_fission_passes(layout, 0, 5)
    with pytest.raises(sph.SphError):
        sph.sph_fission_passes(layout, 3, 1)


def test_fission_passes_known_counts():
    """SoA splits every component; AoS has one substruct; the type split
    separates positions (float64) from the float32 members"""
    soa, aos, shared = sph.LAYOUTS.index("SOA"), sph.LAYOUTS.index("AOS"), sph.LAYOUTS.index("SAOS_SHARED")
    assert len(sph.sph_fission_passes(soa, 2, 1)[0]) == 17
    assert len(sph.sph_fission_passes(aos, 2, 1)[0]) == 1
    assert len(sph.sph_fission_passes(aos, 2, 2)[0]) == 11
    assert sph.sph_fission_passes(aos, 0, 3)[0] == [0x7, 0x88]
    assert len(sph.sph_fission_passes(shared, 2, 1)[0]) == 3
    assert len(sph.sph_fission_passes(shared, 2, 4)[0]) == 4
    assert sph.sph_fission_passes(shared, 0, 1)[1] == [1, 2, 4]


def _status(name, *args):
    return getattr(sph.lib(), name)(*args)


def test_validation_errors_before_any_launch():
    L = sph.lib()
    assert L.sph_status_str(-3).decode() == "buffer too small"
    # null plan
    assert _status("sph_pack", None, 0, None, 0, 1, None, 0, None) == -1
    assert _status("sph_density", None, None, 0, 0, 1, None, None, 0, None, None) == -1
    # unknown layout / loop
    nsub = C.c_int32()
    sb = (C.c_size_t * 32)()
    assert L.sph_layout_info(10, C.byref(nsub), sb) == -2
    assert L.sph_pack_layout(3, C.byref(nsub), (C.c_int32 * 5)(), C.byref(nsub)) == -1
    # plan validation
    ps = inputs.make_config(0, n_side=8, grid=4)
    out = C.c_void_p()
    cells, tasks = ps.cells.copy(), ps.tasks.copy()
    tasks["cj"][5] = 10 ** 6
    assert L.sph_plan_create(cells.ctypes.data, cells.size, tasks.ctypes.data, tasks.size, ps.n,
                             C.byref(out)) == -4
    assert b"out of range" in L.sph_last_error()
    tasks = ps.tasks.copy()
    self_t = np.nonzero(tasks["ci"] == tasks["cj"])[0][0]
    tasks["shift"][self_t] = [1.0, 0, 0]
    assert L.sph_plan_create(cells.ctypes.data, cells.size, tasks.ctypes.data, tasks.size, ps.n,
                             C.byref(out)) == -4
    cells["count"][3] += 10 ** 6
    assert L.sph_plan_create(cells.ctypes.data, cells.size, ps.tasks.ctypes.data, ps.tasks.size, ps.n,
                             C.byref(out)) == -4
    assert L.sph_plan_create(None, -1, None, 0, 0, C.byref(out)) == -1
    assert out.value is None
    # a store whose substruct count does not match its layout
    st = sph.sph_store()
    st.layout, st.nsub, st.n = 0, 3, 10
    assert L.sph_store_put(C.byref(st), 0, C.c_void_p(256), None) == -2
    st.layout = 42
    assert L.sph_store_get(C.byref(st), 0, C.c_void_p(256), None) == -2
    st.layout, st.nsub = 0, 1
    st.sub[0] = 0x1001  # misaligned
    assert L.sph_store_put(C.byref(st), 0, C.c_void_p(256), None) == -1
    assert b"aligned" in L.sph_last_error()
    # conversion: counts must agree and the stores must not overlap
    st.sub[0] = 0x10000
    other = sph.sph_store()
    other.layout, other.nsub, other.n = 0, 1, 11
    other.sub[0] = 0x20000
    assert L.sph_store_convert(C.byref(st), C.byref(other), None) == -1
    assert b"different particle counts" in L.sph_last_error()
    other.n, other.sub[0] = 10, 0x10000 + 0x500   # inside st's 1600 bytes
    assert L.sph_store_convert(C.byref(st), C.byref(other), None) == -1
    assert b"overlaps" in L.sph_last_error()


def test_library_shares_torchs_hip_runtime():
    """Loading the library first must still leave torch's HIP runtime as the
    process's one (both carry the soname libamdhip64.so.7; torch does not run
    on another): a fresh process that loads the library before anything else
    maps only torch's copy."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2606_23891_amd import sph\n"
            "sph.lib()\n"
            "maps = open('/proc/self/maps').read().split()\n"
            "print('\\n'.join(sorted({m for m in maps if 'libamdhip64' in m})))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    mapped = [l for l in out.stdout.split() if l]
    import torch
    torch_lib = os.path.realpath(os.path.join(os.path.dirname(torch.__file__), "lib"))
    assert mapped and all(os.path.realpath(p).startswith(torch_lib) for p in mapped), mapped
