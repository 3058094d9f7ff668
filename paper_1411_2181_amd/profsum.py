"""Summaries of rocprofv3 output for the step kernel.

    python -m paper_1411_2181_amd.profsum trace KERNEL_TRACE.csv [--box 512,256,128]
    python -m paper_1411_2181_amd.profsum traffic FETCH.csv WRITE.csv --precision fp32 \
        [--json profiles/traffic_mv512.json] [--box 512,256,128]
    python -m paper_1411_2181_amd.profsum sq SQ_COUNTERS.csv [--box 512,256,128]

``trace`` groups the dispatches of a ``--kernel-trace`` run by kernel and
launch shape (bx x by x bz, recovered from the grid size and the box: one
workgroup of 2 bx by threads per tile) and prints their mean durations as a
Markdown table.

``traffic`` turns two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
``bench.py --pmc-pass`` into HBM bytes per dispatch.  Each counter is scaled
by what it reads for the pass's reference copy (a 1 GiB device-to-device
copy: 1 GiB read, 1 GiB written), which absorbs the counters' units (on
gfx950 FETCH_SIZE reads about half the bytes a copy moves).  The per-launch
table is merged into a JSON file together with the hash of the kernel sources
it was taken on; bench.py only reports it while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import re
import statistics
from collections import defaultdict

from .build import source_hash

COPY_BYTES = 1 << 30
_STEP = re.compile(r"lbm::k_(step)<[^,]+, [^,]+, (\d+), (\d+)(?:, \w+)*>")


def _launch(kind, bx, by, grid_items, wg_items, box):
    nx, ny, nz = box
    wg = grid_items // wg_items
    cols = -(-nx // bx) * -(-ny // by)
    bz = nz * cols // wg if wg else 0
    return f"{bx}x{by}x{bz}"


def step_dispatches(path, box):
    """(kernel, launch, duration_ns, counter_value or None) per step dispatch."""
    out = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            m = _STEP.search(r["Kernel_Name"])
            if not m:
                continue
            kind, bx, by = m.group(1), int(m.group(2)), int(m.group(3))
            if "Grid_Size" in r:           # counter-collection rows: totals
                grid, wg_items = int(r["Grid_Size"]), int(r["Workgroup_Size"])
            else:                          # kernel-trace rows: per dimension
                grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                wg_items = (int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) *
                            int(r["Workgroup_Size_Z"]))
            key = _launch(kind, bx, by, grid, wg_items, box)
            dur = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            val = float(r["Counter_Value"]) if "Counter_Value" in r else None
            out.append((kind, key, dur, val))
    return out


def copy_reference(path):
    """Counter value of the pass's 1 GiB reference copy (largest copy dispatch)."""
    best = None
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"].lower():
                v = float(r["Counter_Value"])
                if best is None or int(r["Grid_Size"]) > best[0]:
                    best = (int(r["Grid_Size"]), v)
    if best is None:
        raise ValueError(f"no copy dispatch in {path}")
    return best[1]


def trace_table(path, box, tail=0, label=None):
    """Mean durations per (kernel, launch); ``tail`` > 0 keeps only the last
    ``tail`` dispatches of each (bench.py ends with that many eager steps
    timed by HIP events, after the graph-replayed region).  ``label`` names
    the launch of a pinned run (a persistent grid does not encode bz)."""
    groups = defaultdict(list)
    for kind, key, dur, _ in step_dispatches(path, box):
        groups[(kind, label or key)].append(dur)
    rows = []
    for (kind, key), d in groups.items():
        if tail > 0:
            d = d[-tail:]
        rows.append(dict(kernel=f"k_{kind}", launch=key, calls=len(d), mean_us=statistics.mean(d) / 1e3,
                         min_us=min(d) / 1e3, max_us=max(d) / 1e3, total_ms=sum(d) / 1e6))
    rows.sort(key=lambda r: -r["total_ms"])
    return rows


def traffic_table(fetch_csv, write_csv, box):
    """{launch: {kernel: {"fetch": B, "write": B, "bytes": B, "us": mean}}} per dispatch."""
    nodes = box[0] * box[1] * box[2]
    scale = {"fetch": COPY_BYTES / (copy_reference(fetch_csv) * 1024.0),
             "write": COPY_BYTES / (copy_reference(write_csv) * 1024.0)}
    acc = defaultdict(lambda: defaultdict(lambda: defaultdict(list)))
    for which, path in (("fetch", fetch_csv), ("write", write_csv)):
        for kind, key, dur, val in step_dispatches(path, box):
            acc[key][f"k_{kind}"][which].append(val * 1024.0 * scale[which])
            acc[key][f"k_{kind}"]["us"].append(dur / 1e3)
    table = {}
    for key, ks in acc.items():
        ent = {}
        for k, v in ks.items():
            if not v["fetch"] or not v["write"]:
                continue
            f, w = statistics.mean(v["fetch"]), statistics.mean(v["write"])
            ent[k] = dict(fetch=round(f), write=round(w), bytes=round(f + w),
                          bytes_per_node=round((f + w) / nodes, 2), us=round(statistics.mean(v["us"]), 1))
        if "k_step" in ent:
            table[key] = ent
    return table, scale


SQ_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
               "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES")
SIMDS, CLOCK_HZ = 1024, 2.4e9          # MI355X: 256 CUs x 4 SIMDs, 2.4 GHz


def sq_table(path, box):
    """Per step kernel: instructions per lattice node (per-wave counts x 64
    lanes / nodes) and the VALU issue share, the fraction of the SIMDs'
    cycles over the dispatch that its VALU instructions occupy (4 cycles per
    wave64 instruction)."""
    nodes = box[0] * box[1] * box[2]
    acc = defaultdict(lambda: defaultdict(list))
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            m = _STEP.search(r["Kernel_Name"])
            if not m:
                continue
            k = f"k_{m.group(1)}"
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            acc[k]["_dur"].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    rows = []
    for k, c in acc.items():
        mean = {n: statistics.mean(v) for n, v in c.items() if v}
        per = lambda n: mean.get(n, 0.0) * 64.0 / nodes
        dur = mean["_dur"] * 1e-9
        rows.append(dict(kernel=k, valu=per("SQ_INSTS_VALU"), lds=per("SQ_INSTS_LDS"),
                         vmem_rd=per("SQ_INSTS_VMEM_RD"), vmem_wr=per("SQ_INSTS_VMEM_WR"),
                         valu_share=mean.get("SQ_INSTS_VALU", 0.0) * 4.0 / (SIMDS * CLOCK_HZ * dur),
                         wait_frac=mean.get("SQ_WAIT_INST_ANY", 0.0) / max(mean.get("SQ_WAVE_CYCLES", 1.0), 1.0)))
    rows.sort(key=lambda r: r["kernel"])
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--box", default="512,256,128")
    t.add_argument("--tail", type=int, default=0)
    t.add_argument("--launch", default=None, help="label of the pinned launch shape")
    q = sub.add_parser("sq")
    q.add_argument("csv")
    q.add_argument("--box", default="512,256,128")
    p = sub.add_parser("traffic")
    p.add_argument("fetch_csv")
    p.add_argument("write_csv")
    p.add_argument("--precision", required=True)
    p.add_argument("--json")
    p.add_argument("--box", default="512,256,128")
    a = ap.parse_args(argv)
    box = tuple(int(v) for v in a.box.split(","))
    if a.cmd == "trace":
        print("| kernel | launch (bx x by x bz) | calls | mean us | min us | max us |")
        print("|---|---|---|---|---|---|")
        for r in trace_table(a.csv, box, a.tail, a.launch):
            print(f"| {r['kernel']} | {r['launch']} | {r['calls']} | {r['mean_us']:.1f} | "
                  f"{r['min_us']:.1f} | {r['max_us']:.1f} |")
        return 0
    if a.cmd == "sq":
        print("| kernel | VALU / node | LDS / node | VMEM rd / node | VMEM wr / node | VALU issue share | wait / wave cycles |")
        print("|---|---|---|---|---|---|---|")
        for r in sq_table(a.csv, box):
            print(f"| {r['kernel']} | {r['valu']:.0f} | {r['lds']:.1f} | {r['vmem_rd']:.1f} | "
                  f"{r['vmem_wr']:.1f} | {r['valu_share'] * 100:.0f} % | {r['wait_frac'] * 100:.0f} % |")
        return 0
    table, scale = traffic_table(a.fetch_csv, a.write_csv, box)
    print(f"copy-reference scale factors: FETCH_SIZE x{scale['fetch']:.4f}, WRITE_SIZE x{scale['write']:.4f}")
    print("| launch | fetch B/node | write B/node | step B/node | mean us |")
    print("|---|---|---|---|---|")
    nodes = box[0] * box[1] * box[2]
    for key in sorted(table, key=lambda k: table[k]["k_step"]["bytes_per_node"]):
        e = table[key]["k_step"]
        print(f"| {key} | {e['fetch'] / nodes:.1f} | {e['write'] / nodes:.1f} | "
              f"{e['bytes_per_node']} | {e['us']} |")
    if a.json:
        data = {}
        if os.path.exists(a.json):
            with open(a.json) as fh:
                data = json.load(fh)
        data[a.precision] = dict(source_hash=source_hash(), box=list(box),
                                 scale=scale, launches=table)
        with open(a.json, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
