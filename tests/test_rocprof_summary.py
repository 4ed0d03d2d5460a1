"""Host logic behind the bench line's measured fields: the rocprofv3 summary
tool (trace tables, counter averages, HBM bytes scaled by a copy of known
size) and bench.recorded_traffic(), which reports traffic only while the pair
kernel sources hash to the recorded value.  Synthetic trace databases and
counter files stand in for rocprofv3 output."""
import csv
import os
import sqlite3

import pytest

import bench
from paper_1507_07548_amd import rocprof_summary as R


def kernel_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, grid_x int, grid_y int, grid_z int, duration int)")
    con.executemany("insert into kernels values (?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    return path


def counter_csv(path, counter, dispatches):
    """dispatches: (dispatch id, kernel name, grid size, value); each value is
    split over two rows, as rocprofv3 reports one row per agent instance."""
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, grid, value in dispatches:
            for part in (0.25 * value, 0.75 * value):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                            "Counter_Value": part})
    return path


SYM = "void ms2::pair_sym_kernel<float, 1, false, false, true>(ms2::WorkItem const*, int)"
COPY = "__amd_rocclr_copyBuffer"


def test_trace_tables(tmp_path):
    db = kernel_db(str(tmp_path / "k.db"), [
        (SYM, 1000, 1, 1, 4_000_000), (SYM, 1000, 1, 1, 5_000_000),    # two batched launches
        (SYM, 10, 1, 1, 50_000),                                       # a small launch
        ("ms2::md_correct_kernel(int)", 256, 4, 1, 100_000),
    ])
    table = R.summarize(db)
    assert table.splitlines()[2].startswith("| `void ms2::pair_sym_kernel<float, 1, false, false, true>` | 3 |")
    n, avg_us, grid = R.largest_grid(db, "pair_sym_kernel<float")
    assert (n, grid) == (2, 1000) and avg_us == pytest.approx(4500.0)
    sel = R.select(db, ["md_correct", "nothing"]).splitlines()
    assert len(sel) == 3 and "| 1024 | 1 | 100.0 | 0.10 |" in sel[2]
    with pytest.raises(SystemExit):
        R.largest_grid(db, "absent_kernel")


def test_counters_average_the_largest_grid(tmp_path):
    f = counter_csv(str(tmp_path / "c.csv"), "SQ_INSTS_VALU",
                    [(1, SYM, 1000, 300.0), (2, SYM, 1000, 500.0), (3, SYM, 8, 7.0)])
    out = R.counters(f, "pair_sym_kernel<float")
    assert "2 launches of grid 1000" in out and "| SQ_INSTS_VALU | 400 |" in out


def test_traffic_scales_each_counter_by_the_copy(tmp_path, monkeypatch):
    gib = 1 << 30
    # the copy of 1 GiB reads as 0.5 GiB of FETCH_SIZE and 1 GiB of WRITE_SIZE
    fetch = counter_csv(str(tmp_path / "f.csv"), "FETCH_SIZE",
                        [(1, COPY, 4096, gib / 2 / 1024), (2, SYM, 1000, 1000.0), (3, SYM, 1000, 3000.0)])
    write = counter_csv(str(tmp_path / "w.csv"), "WRITE_SIZE",
                        [(1, COPY, 4096, gib / 1024), (2, SYM, 1000, 500.0), (3, SYM, 1000, 500.0)])
    text = R.traffic(fetch, write, gib, "pair_sym_kernel<float")
    # FETCH: 2000 KiB-units x 2048 B; WRITE: 500 x 1024 B
    assert "- hbm_bytes_per_launch: 4.608e+06" in text
    summary = tmp_path / "summary.md"
    summary.write_text("# traffic\n\n" + text + "\n")
    assert bench.recorded(str(summary), "hbm_bytes_per_launch") == pytest.approx(4.608e6)
    # a change of the pair kernel sources voids the record
    monkeypatch.setattr(R, "pair_kernel_source_hash", lambda: "0" * 64)
    assert bench.recorded(str(summary), "hbm_bytes_per_launch") is None
    with pytest.raises(SystemExit):          # no copy of known size in the run
        R.traffic(counter_csv(str(tmp_path / "g.csv"), "FETCH_SIZE", [(2, SYM, 1000, 1.0)]), write, gib,
                  "pair_sym_kernel<float")


def test_source_hash_follows_every_pair_kernel_file(tmp_path, monkeypatch):
    for rel in R.PAIR_SOURCES:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(R.HERE, rel), "rb").read())
    monkeypatch.setattr(R, "HERE", str(tmp_path))
    base = R.pair_kernel_source_hash()
    assert len(base) == 64
    for rel in R.PAIR_SOURCES:
        f = tmp_path / rel
        orig = f.read_bytes()
        f.write_bytes(orig + b" ")
        assert R.pair_kernel_source_hash() != base, rel
        f.write_bytes(orig)
    assert R.pair_kernel_source_hash() == base


def test_gaps_per_step_over_the_last_steps(tmp_path):
    """Three kernels per step with 5 us gaps: over the last three steps, span
    145 us, busy 130 us; a kernel overlapping another (another stream) is
    counted once; the steps before the window are left out."""
    con = sqlite3.connect(str(tmp_path / "g.db"))
    con.execute('create table kernels (name text, start int, "end" int)')
    t, rows = 0, []
    for step in range(5):
        for name, dur in ((SYM, 100_000), ("ms2::reduce_force_kernel", 20_000), ("ms2::md_end", 10_000)):
            rows.append((name, t, t + dur))
            t += dur + 5_000
    rows.append(("overlap", rows[6][1] + 1_000, rows[6][1] + 50_000))    # inside step 2's pair kernel
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    g = R.gaps(str(tmp_path / "g.db"), "pair_sym_kernel", 3)
    assert g["span_us"] == pytest.approx(145.0) and g["busy_us"] == pytest.approx(130.0)
    assert g["idle_frac"] == pytest.approx(15.0 / 145.0)
    with pytest.raises(SystemExit):
        R.gaps(str(tmp_path / "g.db"), "pair_sym_kernel", 5)


def test_flops_weights_each_fp32_counter(tmp_path):
    """FMA counts two operations, ADD, MUL and TRANS one; per wave
    instruction 64 lanes; averaged over the largest-grid launches."""
    names = ["SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_TRANS_F32"]
    path = str(tmp_path / "f.csv")
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, grid, vals in ((1, 1000, (10, 20, 30, 4)), (2, 1000, (10, 20, 30, 4)), (3, 8, (1e6, 0, 0, 0))):
            for name, v in zip(names, vals):
                w.writerow({"Dispatch_Id": d, "Kernel_Name": SYM, "Grid_Size": grid, "Counter_Name": name,
                            "Counter_Value": v})
    out = R.flops(path, "pair_sym_kernel<float", 64.0)
    # (10 + 20 + 2 * 30 + 4) x 64 / 64 pairs = 94 FLOP, (10 + 20 + 30 + 4) = 64 instructions
    assert "- fp32_flop_per_mol_pair_executed: 94.0" in out
    assert "- fp32_instructions_per_mol_pair: 64.0" in out
