"""Summaries of rocprofv3 runs of bench.py, and the HBM traffic figures that
bench.py reports beside its roofline.

HBM traffic per launch comes from two counter runs of the same bench command:
``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` (KiB per dispatch).  Each counter
is scaled by the ratio of a known byte count to what the same counter reads
for a plain elementwise copy of that size (``bench.py --copy-mib``, the
``torch.neg`` over a buffer much larger than the last-level cache), so the
figures are in the copy's bytes.  The summary records a hash of the kernel
sources and the workload; bench.py reports the figures only while both match.

CLI (on the pulled rocprofv3 output directories):
  python -m paper_2606_23891_amd.profiling stats  <kernel_stats.csv> --out F --command C --title T
  python -m paper_2606_23891_amd.profiling traffic <fetch_dir> <write_dir> --copy-mib 1024 \
      --workload W --out F --command-fetch C1 --command-write C2
  python -m paper_2606_23891_amd.profiling sq <pmc_dir> [<pmc_dir> ...] --out F --command C
  python -m paper_2606_23891_amd.profiling layouts <bench_json_line_file> --out F --command C --title T
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_TAG = "neg_kernel"
JSON_BEGIN = "<!-- traffic-json"
JSON_END = "-->"


# translation units no kernel of the step comes from
NOT_STEP = ("sph_adjoint.hip",)


def source_hash() -> str:
    """sha256 over the sources of the step's kernels (every kernel source but
    the adjoint's translation unit) and the build flags"""
    h = hashlib.sha256()
    files = sorted(p for p in glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.hpp"))
                   if os.path.basename(p) not in NOT_STEP)
    files.append(os.path.join(HERE, "build.py"))
    for p in files:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find_csv(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def read_counter(d: str, counter: str):
    """kernel name -> list of per-dispatch values of one counter"""
    path = _find_csv(d, "counter_collection.csv")
    out = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            out[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return dict(out)


def read_counters(d: str):
    """kernel name -> counter -> list of per-dispatch values (every counter of a run)"""
    path = _find_csv(d, "counter_collection.csv")
    out = defaultdict(lambda: defaultdict(list))
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out[row["Kernel_Name"]][row["Counter_Name"]].append(float(row["Counter_Value"]))
    return out


def _mean(v):
    return sum(v) / len(v)


def traffic(fetch_dir: str, write_dir: str, copy_bytes: int) -> dict:
    fe = read_counter(fetch_dir, "FETCH_SIZE")
    wr = read_counter(write_dir, "WRITE_SIZE")
    cf = [k for k in fe if COPY_TAG in k]
    cw = [k for k in wr if COPY_TAG in k]
    if len(cf) != 1 or len(cw) != 1:
        raise RuntimeError(f"calibration copy not found once: {cf} {cw}")
    # the copy reads and writes copy_bytes each; counters are KiB per dispatch
    f_factor = copy_bytes / (_mean(fe[cf[0]]) * 1024.0)
    w_factor = copy_bytes / (_mean(wr[cw[0]]) * 1024.0)
    kern = {}
    for k in sorted(set(fe) & set(wr)):
        if not k.startswith("void sph::") and not k.startswith("sph::"):
            continue
        fb = _mean(fe[k]) * 1024.0 * f_factor
        wb = _mean(wr[k]) * 1024.0 * w_factor
        kern[k] = {"dispatches": len(fe[k]), "fetch_bytes": fb, "write_bytes": wb, "bytes": fb + wb}
    return {"copy_bytes": copy_bytes, "fetch_factor": f_factor, "write_factor": w_factor,
            "copy_fetch_KiB": _mean(fe[cf[0]]), "copy_write_KiB": _mean(wr[cw[0]]), "kernels": kern}


def traffic_markdown(t: dict, workload: str, cmd_fetch: str, cmd_write: str, algo: dict | None = None) -> str:
    t = dict(t, workload=workload, source_hash=source_hash())
    lines = [f"# HBM traffic per launch: {workload}", "",
             "Two counter runs of the same bench command (one counter each), on one MI355X from the "
             "repository root:", "", "```", cmd_fetch, cmd_write, "```", "",
             f"Calibration: one plain elementwise copy of {t['copy_bytes']} bytes (read and write) reads "
             f"FETCH_SIZE {t['copy_fetch_KiB']:.0f} KiB and WRITE_SIZE {t['copy_write_KiB']:.0f} KiB; "
             f"factors {t['fetch_factor']:.4f} (fetch) and {t['write_factor']:.4f} (write) scale every "
             "kernel's counters below.", "",
             "| kernel | dispatches | fetch MB | write MB | total MB |" + (" algorithmic MB | ratio |" if algo else ""),
             "|---|---|---|---|---|" + ("---|---|" if algo else "")]
    for k, v in sorted(t["kernels"].items(), key=lambda kv: -kv[1]["bytes"]):
        row = (f"| `{k}` | {v['dispatches']} | {v['fetch_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
               f"{v['bytes'] / 1e6:.1f} |")
        if algo:
            a = algo.get(k)
            row += f" {a / 1e6:.1f} | {v['bytes'] / a:.2f} |" if a else " | |"
        lines.append(row)
    lines += ["", f"Kernel sources hash {t['source_hash']}.", "", JSON_BEGIN, json.dumps(t), JSON_END, ""]
    return "\n".join(lines)


def load_traffic(path: str, workload: str):
    """the traffic summary at path if it matches these sources and workload, else None"""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    i = txt.find(JSON_BEGIN)
    if i < 0:
        return None
    j = txt.find(JSON_END, i)
    try:
        t = json.loads(txt[i + len(JSON_BEGIN):j])
    except ValueError:
        return None
    if t.get("source_hash") != source_hash() or t.get("workload") != workload:
        return None
    return t


def stats_markdown(stats_csv: str, title: str, command: str, note: str = "") -> str:
    rows = list(csv.DictReader(open(stats_csv, newline="")))
    lines = [f"# {title}", "", "Command (run on one MI355X from the repository root):", "", "```", command, "```", ""]
    if note:
        lines += [note, ""]
    lines += ["| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"]
        if len(name) > 70:
            name = name[:67] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines) + "\n"


def sq_markdown(dirs, title: str, commands, match: str = "sph::") -> str:
    """per-kernel averages of every counter in one or more --pmc runs"""
    table = defaultdict(dict)
    names = []
    for d in dirs:
        for k, cs in read_counters(d).items():
            if match not in k:
                continue
            for c, v in cs.items():
                table[k][c] = _mean(v)
                if c not in names:
                    names.append(c)
    lines = [f"# {title}", "", "Commands (each a run of its own, on one MI355X from the repository root):", "",
             "```", *commands, "```", "", "Per-dispatch averages.", ""]
    for k in sorted(table):
        lines.append(f"## `{k}`")
        lines.append("")
        lines.append("| counter | value |")
        lines.append("|---|---|")
        for c in names:
            if c in table[k]:
                lines.append(f"| {c} | {table[k][c]:.6g} |")
        lines.append("")
    return "\n".join(lines)


def layouts_markdown(bench_out: str, title: str, command: str) -> str:
    """the per-layout pack / unpack table, the offload table and the conversion
    table of one bench.py run (its JSON line)"""
    with open(bench_out) as f:
        d = json.loads([ln for ln in f.read().splitlines() if ln.strip().startswith("{")][-1])
    lines = [f"# {title}", "", "Command (one MI355X, repository root):", "", "```", command, "```", ""]
    if "layouts" in d:
        lines += ["Per-loop form (each loop packed, then unpacked into the store), batched, tuned launch "
                  "parameters; HIP-event averages per layout.  GB/s are algorithmic bytes (fields the loop "
                  "needs + packed record; results + outputs), so AoS is charged only for the bytes it needs.", "",
                  "| layout | pack d | unpack d | pack g | unpack g | pack f | unpack f | total ms | vs AoS |",
                  "|---|---|---|---|---|---|---|---|---|"]
        for name, r in d["layouts"].items():
            cells = []
            for loop in ("density", "gradient", "force"):
                x = r[loop]
                cells.append(f"{x['pack_ms']:.3f} ms ({x['pack_GB/s']:.0f} GB/s)")
                cells.append(f"{x['unpack_ms']:.3f} ms ({x['unpack_GB/s']:.0f} GB/s)")
            lines.append(f"| {name} | " + " | ".join(cells) + f" | {r['total_ms']:.3f} | {r.get('vs_AOS', 0):.3f} |")
        lines.append("")
        if any("staged" in r for r in d["layouts"].values()):
            lines += ["Staged step (the form the benchmark's step runs): the three packs, each taking the "
                      "step's earlier outputs from its result planes, writing the derived planes and, where it "
                      "loads an output's record whole, storing that output; then the write-back of the rest.  "
                      "GB/s on the same algorithmic bytes as the step's stages.", "",
                      "| layout | pack d | pack g | pack f | write-back | total ms |", "|---|---|---|---|---|---|"]
            for name, r in d["layouts"].items():
                g = r.get("staged")
                if not g:
                    continue
                cells = [f"{g[k]['ms']:.3f} ms ({g[k]['GB/s']:.0f} GB/s)"
                         for k in ("pack_density", "pack_gradient", "pack_force", "writeback")]
                lines.append(f"| {name} | " + " | ".join(cells) + f" | {g['total_ms']:.3f} |")
            lines.append("")
    if "offload" in d:
        lines += ["Offload form (host store in pinned memory; per loop, H2D of the substructs the loop reads or "
                  "partially writes, batched compute, D2H of the substructs holding its outputs); pipelined: "
                  "`sph_offload_step_async` with 4 and 16 bundles of cells, every input substruct sent once per "
                  "step:", "",
                  "| layout | ms/step | H2D GB | D2H GB | link GB/s | pipelined, 4 bundles | pipelined, 16 bundles |",
                  "|---|---|---|---|---|---|---|"]
        for name, r in d["offload"].items():
            if not isinstance(r, dict):
                continue
            lines.append(f"| {name} | {r['ms_per_step']:.1f} | {r['h2d_GB']:.2f} | {r['d2h_GB']:.2f} | "
                         f"{r['link_GB/s']:.1f} | {r['async4_ms_per_step']:.1f} | {r['async16_ms_per_step']:.1f} |")
        if "pinned_copy_h2d_GB/s" in d["offload"]:
            lines += ["", f"Pinned hipMemcpy H2D: {d['offload']['pinned_copy_h2d_GB/s']} GB/s."]
        lines.append("")
    if "convert" in d:
        lines += ["Whole-store layout conversion (`sph_store_convert`; bytes = every record of both stores once):",
                  "", "| conversion | ms | GB moved | GB/s |", "|---|---|---|---|"]
        for name, r in d["convert"].items():
            lines.append(f"| {name.replace('->', '→')} | {r['ms']:.3f} | {r['bytes'] / 1e9:.2f} | {r['GB/s']:.0f} |")
        lines.append("")
    lines += [f"Same run: staged batched step {d['ms_per_step']:.2f} ms ({d['value']:.3e} pairs/s).", ""]
    return "\n".join(lines)


def fission_markdown(bench_out: str, title: str, command: str) -> str:
    """the loop-fission table of one bench.py --fission run (its JSON line):
    pack + unpack per step for every schedule, then each loop's pack and
    unpack times"""
    with open(bench_out) as f:
        d = json.loads([ln for ln in f.read().splitlines() if ln.strip().startswith("{")][-1])
    fis = d["fission"]
    scheds = list(next(iter(fis.values())).keys())
    label = lambda k: k.replace("_", " ")
    lines = [f"# {title}", "", "Command (one MI355X, repository root):", "", "```", command, "```", "",
             "`sph_tuning.pack_schedule` per column; each group of members (`sph_fission_passes`) is its own "
             "kernel launch.",
             "Entries: pack + unpack of all three loops per step, ms (relative to the fused kernels; pack + "
             "unpack kernel launches).", "",
             "| layout | " + " | ".join(label(k) for k in scheds) + " |",
             "|---|" + "---|" * len(scheds)]
    for name, rows in fis.items():
        cells = []
        for k in scheds:
            r = rows[k]
            npk = sum(v[0] for v in r["kernels"].values())
            nup = sum(v[1] for v in r["kernels"].values())
            cells.append(f"{r['total_ms']:.3f} ({r['vs_by_particle']:.2f}×; {npk}+{nup})")
        lines.append(f"| {name} | " + " | ".join(cells) + " |")
    lines += ["", "Per loop (pack ms / unpack ms):", "", "| layout | schedule | density | gradient | force |",
              "|---|---|---|---|---|"]
    for name, rows in fis.items():
        for k in scheds:
            r = rows[k]
            cells = [f"{r[lp]['pack_ms']:.3f} / {r[lp]['unpack_ms']:.3f}" for lp in ("density", "gradient", "force")]
            lines.append(f"| {name} | {label(k)} | " + " | ".join(cells) + " |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--out", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command-fetch", required=True)
    t.add_argument("--command-write", required=True)
    t.add_argument("--algo", default=None, help="JSON file: kernel name -> algorithmic bytes per launch")
    q = sub.add_parser("sq")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--out", required=True)
    q.add_argument("--title", required=True)
    q.add_argument("--command", action="append", required=True)
    fz = sub.add_parser("fission")
    fz.add_argument("bench_out")
    fz.add_argument("--out", required=True)
    fz.add_argument("--title", required=True)
    fz.add_argument("--command", required=True)
    y = sub.add_parser("layouts")
    y.add_argument("bench_out")
    y.add_argument("--out", required=True)
    y.add_argument("--title", required=True)
    y.add_argument("--command", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        txt = stats_markdown(a.csv, a.title, a.command, a.note)
    elif a.cmd == "traffic":
        algo = json.load(open(a.algo)) if a.algo else None
        txt = traffic_markdown(traffic(a.fetch_dir, a.write_dir, a.copy_mib << 20), a.workload,
                               a.command_fetch, a.command_write, algo)
    elif a.cmd == "layouts":
        txt = layouts_markdown(a.bench_out, a.title, a.command)
    elif a.cmd == "fission":
        txt = fission_markdown(a.bench_out, a.title, a.command)
    else:
        txt = sq_markdown(a.dirs, a.title, a.command)
    with open(a.out, "w") as f:
        f.write(txt)
    print(f"wrote {a.out}")


if __name__ == "__main__":
    main()
