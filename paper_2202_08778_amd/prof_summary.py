"""Text summaries of rocprofv3 runs of bench.py, for the committed profile records.

  trace:  per-kernel dispatch counts and durations from a --kernel-trace CSV;
  hbm:    per-kernel HBM bytes per dispatch from a FETCH_SIZE pass and a WRITE_SIZE pass
          (counter_collection CSVs), each scaled by what the same counter reads for the run's plain
          device copies of 256 MiB (bench.py --copy-calibration), grouped into the library's kernel
          classes; also a JSON record that bench.py reads for its roofline's traffic, tied to the
          kernel sources by their hash;
  insts:  instruction counts per dispatch and per cell of the fine-grid stencil kernels from one SQ counter
          pass (counter_collection CSV), with the VALU issue floor at one wave-instruction per clock per CU.

Kernels are told apart by name and grid size; an apply sweep whose grid is smaller than the largest
one is a multigrid coarse level.

  python -m paper_2202_08778_amd.prof_summary trace TRACE_CSV OUT_MD --cmd CMD --title TITLE
  python -m paper_2202_08778_amd.prof_summary hbm FETCH_CSV WRITE_CSV OUT_MD OUT_JSON --n N --cmds CMD...
  python -m paper_2202_08778_amd.prof_summary insts PMC_CSV OUT_MD --cells CELLS --cmd CMD --title TITLE
"""
import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# the sources bench.py hashes to decide whether a traffic record still describes the kernels
HASHED = ("rad_single.hip", "rad_device.h", "rad_apply_tiled.h", "rad_amr.h")
COPY_BYTES = 256 * 1024 * 1024


def short_name(name):
    name = name.replace("(anonymous namespace)::", "").replace("void ", "").replace("vr::", "")
    return re.split(r"\((?!anonymous)", name)[0].strip()


def grid_of(r):
    for k in ("Grid_Size", "Grid_Size_X", "Grid_X"):
        if r.get(k):
            return int(r[k])
    return 0


def kernel_class(name, grid, fine_grid):
    if name.startswith("k_apply_tiled"):
        return "apply_fp32" if grid >= fine_grid else "multigrid_levels"
    for prefix, cls in (("k_mg_average", "setup"), ("k_mg_face", "setup"), ("k_mg_", "multigrid_levels"),
                        ("k_residual", "residual_fp64"), ("k_multidot", "multidot_fp32"),
                        ("k_orth_update", "orth_update_fp32"), ("k_update_x", "update_x_fp32"),
                        ("k_combine", "update_x_fp32"), ("k_exchange", "exchange_fp64"), ("k_commit", "commit"),
                        ("k_setup", "setup"), ("k_face_coef", "setup"), ("k_closure", "closure")):
        if name.startswith(prefix):
            return cls
    return None


def trace(args):
    agg = collections.defaultdict(lambda: [0, 0.0, float("inf"), 0.0])
    for r in csv.DictReader(open(args.csv)):
        key = (short_name(r["Kernel_Name"]), grid_of(r))
        dt = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg[key]
        a[0] += 1
        a[1] += dt
        a[2] = min(a[2], dt)
        a[3] = max(a[3], dt)
    tot = sum(a[1] for a in agg.values())
    lines = [f"# {args.title}", "", "Command (repository root):", "", f"    {args.cmd}", "",
             f"Kernel time in the run: {tot / 1e3:.1f} ms over {sum(a[0] for a in agg.values())} dispatches.", "",
             "| kernel | grid (threads) | dispatches | total ms | share | mean us | min us | max us |",
             "|---|---|---|---|---|---|---|---|"]
    for (k, g), (n, t, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:args.top]:
        lines.append(f"| {k} | {g} | {n} | {t / 1e3:.2f} | {100 * t / tot:.1f}% | {t / n:.1f} | {lo:.1f} | {hi:.1f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def counters(path, counter):
    """Per (kernel, grid): dispatches and summed counter; and the counter of the calibration copies,
    the run's last four device-copy dispatches (bench.py makes them after everything else)."""
    per = collections.defaultdict(lambda: [0, 0.0])
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        name, g, v = short_name(r["Kernel_Name"]), grid_of(r), float(r["Counter_Value"])
        if "copyBuffer" in name:
            copies.append((int(r["Dispatch_Id"]), v))
        per[(name, g)][0] += 1
        per[(name, g)][1] += v
    last = [v for _, v in sorted(copies)[-4:]]
    return per, sum(last) / len(last)


def hbm(args):
    fetch, fcopy = counters(args.fetch, "FETCH_SIZE")
    write, wcopy = counters(args.write, "WRITE_SIZE")
    fc, wc = fcopy, wcopy   # KiB per calibration copy
    rs, ws = COPY_BYTES / (fc * 1024), COPY_BYTES / (wc * 1024)
    fine = max(g for (k, g) in fetch if k.startswith("k_apply_tiled"))
    rows, cls = [], collections.defaultdict(lambda: [0, 0.0, 0.0])
    kernels = {}
    for key in sorted(fetch, key=lambda k: -fetch[k][1]):
        k, g = key
        c = kernel_class(k, g, fine)
        if c is None:
            continue
        n, fkib = fetch[key]
        wn, wkib = write.get(key, (n, 0.0))
        rb, wb = rs * 1024 * fkib / n, ws * 1024 * wkib / max(wn, 1)
        rows.append(f"| {k} | {g} | {c} | {n} | {fkib / n:.0f} | {wkib / max(wn, 1):.0f} | {rb / 1e6:.1f} | {wb / 1e6:.1f} |")
        kernels[f"{k} [grid {g}]"] = {"read_bytes": rb, "write_bytes": wb, "dispatches": n, "class": c}
        cl = cls[c]
        cl[0] += n
        cl[1] += rb * n
        cl[2] += wb * n
    classes = {c: {"read_bytes": v[1] / v[0], "write_bytes": v[2] / v[0], "dispatches": v[0]} for c, v in cls.items()}
    lines = [f"# {args.title}: HBM bytes per dispatch", "", "Commands (two passes, repository root):", ""]
    lines += [f"    {c}" for c in args.cmds]
    lines += ["", f"Calibration: a plain device copy of 256 MiB reads {fc:.0f} KiB FETCH_SIZE and {wc:.0f} KiB "
                  f"WRITE_SIZE per dispatch: read scale {rs:.3f}, write scale {ws:.3f}.  Scaled values are bytes "
                  "per dispatch.", "",
              "| kernel | grid (threads) | class | dispatches | FETCH KiB/disp (raw) | WRITE KiB/disp (raw) | "
              "scaled read MB | scaled write MB |", "|---|---|---|---|---|---|---|---|"] + rows
    lines += ["", "Per kernel class (dispatch-weighted), scaled bytes per dispatch:", "",
              "| class | dispatches | read MB | write MB |", "|---|---|---|---|"]
    for c, v in sorted(classes.items()):
        lines.append(f"| {c} | {v['dispatches']} | {v['read_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} |")
    open(args.out_md, "w").write("\n".join(lines) + "\n")
    src = b"".join(open(os.path.join(HERE, "csrc", f), "rb").read() for f in HASHED)
    rec = {"source_sha256": hashlib.sha256(src).hexdigest(), "workload": args.title, "n": args.n,
           "commands": args.cmds, "read_scale": rs, "write_scale": ws, "kernels": kernels, "classes": classes}
    json.dump(rec, open(args.out_json, "w"), indent=1)


def insts(args):
    """Per fine-grid stencil kernel (the largest grid of k_apply_tiled, and k_residual_tiled at that grid):
    the mean over dispatches of each device-wide SQ counter, and per cell: the count x 64 / cells, i.e. the
    instructions of the wave that holds the cell (one cell per lane)."""
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    ids = collections.defaultdict(set)
    rows = list(csv.DictReader(open(args.csv)))
    fine = max(grid_of(r) for r in rows if short_name(r["Kernel_Name"]).startswith("k_apply_tiled"))
    for r in rows:
        k, g = short_name(r["Kernel_Name"]), grid_of(r)
        if g != fine or not k.startswith(("k_apply_tiled", "k_residual_tiled")):
            continue
        per[k][r["Counter_Name"]] += float(r["Counter_Value"])
        ids[k].add(r["Dispatch_Id"])
    names = ("SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR")
    lines = [f"# {args.title}: instruction counters", "", "Command (repository root):", "", f"    {args.cmd}", "",
             f"Per dispatch: the mean over the run's dispatches of each fine-grid kernel ({fine} threads) of the "
             "counter summed over the device.  Per cell: that count x 64 / "
             f"{args.cells} cells (the instructions of the wave that holds the cell, one cell per lane).  VALU "
             f"floor: the VALU count / ({args.cus} CUs x 1 wave-instruction per clock x {args.ghz} GHz), four "
             "16-lane SIMDs per CU taking 4 clocks per wave64 instruction.", "",
             "| kernel | dispatches | waves | VALU / dispatch | VALU / cell | LDS / cell | SALU / cell | VMEM rd / cell | "
             "VMEM wr / cell | VALU floor us |", "|---|---|---|---|---|---|---|---|---|---|"]
    for k in sorted(per, key=lambda k: -per[k]["SQ_INSTS_VALU"] / len(ids[k])):
        n = len(ids[k])
        m = {c: per[k][c] / n for c in per[k]}
        pc = [f"{m.get(c, 0.0) * 64 / args.cells:.1f}" for c in names]
        floor = m.get("SQ_INSTS_VALU", 0.0) / (args.cus * args.ghz * 1e9) * 1e6
        lines.append(f"| {k} | {n} | {m.get('SQ_WAVES', 0):.0f} | {m.get('SQ_INSTS_VALU', 0):.4g} | " + " | ".join(pc) +
                     f" | {floor:.1f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--top", type=int, default=30)
    h = sub.add_parser("hbm")
    h.add_argument("fetch")
    h.add_argument("write")
    h.add_argument("out_md")
    h.add_argument("out_json")
    h.add_argument("--n", type=int, required=True)
    h.add_argument("--title", required=True)
    h.add_argument("--cmds", nargs="+", required=True)
    i = sub.add_parser("insts")
    i.add_argument("csv")
    i.add_argument("out")
    i.add_argument("--cells", type=int, required=True)
    i.add_argument("--cmd", required=True)
    i.add_argument("--title", required=True)
    i.add_argument("--cus", type=int, default=256)
    i.add_argument("--ghz", type=float, default=2.4)
    args = ap.parse_args()
    {"trace": trace, "hbm": hbm, "insts": insts}[args.mode](args)


if __name__ == "__main__":
    main()
