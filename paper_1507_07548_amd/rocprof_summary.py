"""Short text summaries of rocprofv3 output.

  kernels <results.db> [kernel substring]
      per-kernel calls, average and total duration from a --kernel-trace
      results database; with a substring, also the average duration of that
      kernel's largest-grid (batched) launches.
  counters <counters.csv> <kernel substring>
      every counter of a --pmc run per launch, averaged over the
      largest-grid dispatches whose name holds the substring.
  select <results.db> <substring;substring;...>
      per kernel and grid size, calls and durations of the kernels whose
      name holds one of the ';'-separated substrings.
  gaps <results.db> <marker substring> <steps>
      device idle time between kernels over the last <steps> steps of a
      run: a step starts at a dispatch of the marker kernel (one per step);
      prints per step the span, the kernels' busy time and the idle rest.
  flops <f32.csv> <kernel substring> <molecule pairs per launch>
      executed FP32 FLOP per molecule pair of the largest-grid launches from
      a --pmc run of SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F32 (per wave
      instruction: 64 lanes; an FMA counts 2); prints the field bench.py reads.
  traffic <fetch.csv> <write.csv> <copy_bytes> <kernel substring>
      HBM bytes per launch of the largest-grid dispatches whose name holds
      the substring, from two --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per
      dispatch).  Each counter is scaled by bytes / counter of the largest
      device-to-device copy in the same run (a copy of copy_bytes bytes reads
      and writes exactly that many).  Prints the fields bench.py reads.
"""
import csv
import hashlib
import os
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PAIR_SOURCES = ["csrc/forces.hip", "csrc/pair_math.h", "csrc/internal.h", "csrc/site_frame.h", "csrc/quat.h",
                "csrc/kspace_sums.h"]


def pair_kernel_source_hash():
    """sha256 over the sources of the pair kernels (a changed kernel voids
    counters taken before the change)."""
    h = hashlib.sha256()
    for rel in PAIR_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def summarize(db_path, top=12):
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, count(*), avg(duration), sum(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    total = sum(r[3] for r in rows)
    out = ["| kernel | calls | avg us | total ms | % time |", "|---|---|---|---|---|"]
    for name, calls, avg, tot in rows[:top]:
        out.append(f"| `{name.split('(')[0]}` | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.2f} | {100 * tot / total:.1f} |")
    return "\n".join(out)


def largest_grid(db_path, substring):
    """Calls and average duration (us) of the largest-grid dispatches of the
    kernels whose name holds the substring (the batched launches)."""
    con = sqlite3.connect(db_path)
    rows = con.execute("select grid_x * grid_y * grid_z, duration from kernels where name like ?",
                       (f"%{substring}%",)).fetchall()
    if not rows:
        raise SystemExit(f"no dispatch of a kernel named like {substring!r}")
    gmax = max(g for g, _ in rows)
    d = [t for g, t in rows if g == gmax]
    return len(d), sum(d) / len(d) / 1e3, gmax


def select(db_path, substrings):
    """Per kernel and grid size, for the kernels whose name holds one of the
    substrings: calls, average and total duration."""
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, grid_x * grid_y * grid_z, count(*), avg(duration), sum(duration) "
                       "from kernels group by name, grid_x * grid_y * grid_z").fetchall()
    out = ["| kernel | grid (work-items) | calls | avg us | total ms |", "|---|---|---|---|---|"]
    for name, grid, calls, avg, tot in sorted(rows, key=lambda r: -r[4]):
        if any(sub in name for sub in substrings):
            out.append(f"| `{name.split('(')[0]}` | {grid} | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.2f} |")
    return "\n".join(out)


def _kernel_intervals(con):
    cols = [r[1] for r in con.execute("pragma table_info(kernels)")]
    for a, b in (("start", "end"), ("start_ns", "end_ns"), ("begin", "end")):
        if a in cols and b in cols:
            return con.execute(f'select name, "{a}", "{b}" from kernels order by "{a}"').fetchall()
    raise SystemExit(f"kernels table without start/end columns: {cols}")


def gaps(db_path, marker, steps):
    """Per step over the last `steps` steps: span (first marker dispatch of a
    step to the next one's), summed kernel time inside it (overlaps merged)
    and the idle rest, in microseconds."""
    con = sqlite3.connect(db_path)
    rows = _kernel_intervals(con)
    starts = [a for n, a, _ in rows if marker in n]
    if len(starts) < steps + 1:
        raise SystemExit(f"fewer than {steps + 1} dispatches of {marker!r}")
    t0, t1 = starts[-steps - 1], starts[-1]
    busy, cur_a, cur_b = 0, None, None
    for _, a, b in rows:
        a, b = max(a, t0), min(b, t1)
        if b <= a:
            continue
        if cur_b is None or a > cur_b:
            if cur_b is not None:
                busy += cur_b - cur_a
            cur_a, cur_b = a, b
        else:
            cur_b = max(cur_b, b)
    if cur_b is not None:
        busy += cur_b - cur_a
    per = [(t1 - t0) / steps / 1e3, busy / steps / 1e3]
    n_k = sum(1 for _, a, b in rows if a >= t0 and a < t1)
    return {"span_us": per[0], "busy_us": per[1], "idle_us": per[0] - per[1],
            "idle_frac": 1.0 - per[1] / per[0], "kernels_per_step": n_k / steps}


def _dispatches(csv_path, counter):
    """{dispatch id: (kernel name, grid size, counter value)}"""
    out = {}
    with open(csv_path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            d = out.get(r["Dispatch_Id"])
            v = float(r["Counter_Value"]) + (d[2] if d else 0.0)
            out[r["Dispatch_Id"]] = (r["Kernel_Name"], int(r["Grid_Size"]), v)
    return out


def _per_launch(disp, substring):
    hits = [(g, v, n) for n, g, v in disp.values() if substring in n]
    if not hits:
        raise SystemExit(f"no dispatch of a kernel named like {substring!r}")
    gmax = max(g for g, _, _ in hits)
    vals = [v for g, v, _ in hits if g == gmax]
    return sum(vals) / len(vals), len(vals), hits[0][2].split("(")[0]


def _copy_kib(disp):
    copies = [v for n, g, v in disp.values() if "copy" in n.lower()]
    if not copies:
        raise SystemExit("no copy kernel in the run: pass --copy-calibration-mib to bench.py")
    return max(copies)


def counters(csv_path, substring):
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if substring not in r["Kernel_Name"]:
            continue
        d = per.setdefault(r["Dispatch_Id"], [int(r["Grid_Size"]), r["Kernel_Name"].split("(")[0], {}])
        d[2][r["Counter_Name"]] = d[2].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no dispatch of a kernel named like {substring!r}")
    gmax = max(d[0] for d in per.values())
    big = [d for d in per.values() if d[0] == gmax]
    names = sorted(big[0][2])
    lines = [f"Kernel `{big[0][1]}`: {len(big)} launches of grid {gmax} work-items.", "",
             "| counter | per launch |", "|---|---|"]
    for k in names:
        lines.append(f"| {k} | {sum(d[2][k] for d in big) / len(big):.6g} |")
    return "\n".join(lines)


def flops(csv_path, substring, mol_pairs):
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if substring not in r["Kernel_Name"]:
            continue
        d = per.setdefault(r["Dispatch_Id"], [int(r["Grid_Size"]), {}])
        d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    if not per:
        raise SystemExit(f"no dispatch of a kernel named like {substring!r}")
    gmax = max(d[0] for d in per.values())
    big = [d[1] for d in per.values() if d[0] == gmax]
    avg = {k: sum(b.get(k, 0.0) for b in big) / len(big) for k in big[0]}
    w = {"SQ_INSTS_VALU_ADD_F32": 1, "SQ_INSTS_VALU_MUL_F32": 1, "SQ_INSTS_VALU_FMA_F32": 2,
         "SQ_INSTS_VALU_TRANS_F32": 1}
    missing = [k for k in w if k not in avg]
    if missing:
        raise SystemExit(f"counters missing: {missing}")
    lanes = 64.0
    flop = sum(w[k] * avg[k] for k in w) * lanes
    inst = sum(avg[k] for k in w) * lanes
    lines = [f"{len(big)} launches of grid {gmax} work-items; {mol_pairs:.6g} molecule pairs per launch.", "",
             "| counter | per launch | per molecule pair (x 64 lanes) |", "|---|---|---|"]
    for k in sorted(w):
        lines.append(f"| {k} | {avg[k]:.6g} | {avg[k] * lanes / mol_pairs:.1f} |")
    lines += ["", f"- fp32_instructions_per_mol_pair: {inst / mol_pairs:.1f}",
              f"- fp32_flop_per_mol_pair_executed: {flop / mol_pairs:.1f}",
              f"- source_sha256: `{pair_kernel_source_hash()}`"]
    return "\n".join(lines)


def traffic(fetch_csv, write_csv, copy_bytes, substring):
    fd, wd = _dispatches(fetch_csv, "FETCH_SIZE"), _dispatches(write_csv, "WRITE_SIZE")
    f_kib, nf, name = _per_launch(fd, substring)
    w_kib, nw, _ = _per_launch(wd, substring)
    cf, cw = _copy_kib(fd), _copy_kib(wd)
    sf, sw = copy_bytes / cf, copy_bytes / cw            # bytes per counter unit, per direction
    total = f_kib * sf + w_kib * sw
    lines = [
        f"Kernel `{name}`: {nf} (FETCH_SIZE) and {nw} (WRITE_SIZE) batched launches.",
        "",
        "| | counter per launch (KiB) | copy of known size (KiB) | bytes per unit | HBM bytes per launch |",
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {f_kib:.1f} | {cf:.1f} | {sf:.2f} | {f_kib * sf:.4g} |",
        f"| WRITE_SIZE | {w_kib:.1f} | {cw:.1f} | {sw:.2f} | {w_kib * sw:.4g} |",
        "",
        f"- hbm_bytes_per_launch: {total:.6g}",
        f"- source_sha256: `{pair_kernel_source_hash()}`",
    ]
    return "\n".join(lines)


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "counters":
        print(counters(sys.argv[2], sys.argv[3]))
    elif len(sys.argv) >= 2 and sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5]))
    elif len(sys.argv) >= 2 and sys.argv[1] == "flops":
        print(flops(sys.argv[2], sys.argv[3], float(sys.argv[4])))
    elif len(sys.argv) >= 2 and sys.argv[1] == "gaps":
        g = gaps(sys.argv[2], sys.argv[3], int(sys.argv[4]))
        print(f"per step over the last {sys.argv[4]} steps: span {g['span_us']:.1f} us, kernels busy "
              f"{g['busy_us']:.1f} us, idle {g['idle_us']:.1f} us ({100 * g['idle_frac']:.1f} %), "
              f"{g['kernels_per_step']:.1f} kernels per step")
    elif len(sys.argv) >= 2 and sys.argv[1] == "select":
        print(select(sys.argv[2], sys.argv[3].split(";")))
    elif len(sys.argv) >= 2 and sys.argv[1] == "kernels":
        print(summarize(sys.argv[2]))
        if len(sys.argv) >= 4:
            n, avg, g = largest_grid(sys.argv[2], sys.argv[3])
            print(f"\nLargest-grid launches of `{sys.argv[3]}` (grid {g} work-items): {n} calls, "
                  f"average {avg:.1f} us.")
    else:
        print(summarize(sys.argv[1]))
