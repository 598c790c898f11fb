"""Host logic of the rocprofv3 summaries (paper_1607_02904_amd.profsum) on
small synthetic trace files: no GPU, no profiler."""
import csv

from paper_1607_02904_amd import profsum

FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]


def _trace(path, rows):
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=FIELDS)
        wr.writeheader()
        for name, t0, dur_ns in rows:
            wr.writerow({"Kernel_Name": name, "Start_Timestamp": t0, "End_Timestamp": t0 + dur_ns})


def test_tail_takes_the_last_dispatches_of_each_kernel(tmp_path):
    # kernel A: two slow tuning launches, then three timed ones of 10, 20, 30 us;
    # kernel B: one launch of 5 us; kernel C is filtered out
    rows = [("k_a<1>", 0, 900_000), ("k_a<1>", 1_000_000, 800_000),
            ("k_a<1>", 2_000_000, 10_000), ("k_a<1>", 3_000_000, 20_000),
            ("k_a<1>", 4_000_000, 30_000), ("k_b", 2_500_000, 5_000), ("other", 10, 1_000)]
    p = tmp_path / "trace.csv"
    _trace(p, rows)
    lines = profsum.tail(str(p), ["k_"], 3)
    assert len(lines) == 2
    assert lines[0].startswith("k_a<1>")  # largest total time first
    f = lines[0].split()
    assert f[f.index("dispatches") + 1] == "3"
    assert float(f[f.index("avg_us") + 1]) == 20.0
    assert float(f[f.index("min_us") + 1]) == 10.0
    assert float(f[f.index("max_us") + 1]) == 30.0
    g = lines[1].split()
    assert g[0] == "k_b" and float(g[g.index("avg_us") + 1]) == 5.0


def test_tail_orders_by_start_time_not_by_file_order(tmp_path):
    rows = [("k_a", 3_000_000, 30_000), ("k_a", 1_000_000, 900_000), ("k_a", 2_000_000, 10_000)]
    p = tmp_path / "trace.csv"
    _trace(p, rows)
    (line,) = profsum.tail(str(p), [], 2)
    f = line.split()
    assert float(f[f.index("avg_us") + 1]) == 20.0  # the launches at t = 2 and 3 ms


def test_rebuild_splits_the_list_kernels_by_step(tmp_path):
    # two MD steps: the first rebuilds (k_build 50 us), the second does not
    # (every list kernel returns at once); each chain ends at the force kernel
    t = 0
    rows = []
    for build_us in (50, 2):
        for name, us in (("k_bin", 10 if build_us > 8 else 1), ("k_cells", 20 if build_us > 8 else 1),
                         ("k_build<true, false, 256>", build_us), ("k_slots", 12 if build_us > 8 else 1),
                         ("k_reverse", 30 if build_us > 8 else 1), ("k_force_wave<float>", 80),
                         ("k_vv_gather_kick_drift<float, true>", 18)):
            rows.append(("void ters::(anonymous namespace)::%s(int)" % name, t, us * 1000))
            t += 100_000
    p = tmp_path / "trace.csv"
    _trace(p, rows)
    out = profsum.rebuild(str(p), 8.0)
    n, per, total = out["rebuild"]
    assert n == 1 and per["k_build"] == 50.0 and per["k_reverse"] == 30.0
    assert total == 10 + 20 + 50 + 12 + 30
    n, per, total = out["no_rebuild"]
    assert n == 1 and total == 1 + 1 + 2 + 1 + 1


def _counters(path, rows):
    fields = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        wr = csv.DictWriter(f, fieldnames=fields)
        wr.writeheader()
        for d, name, grid, counter, value in rows:
            wr.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid,
                         "Counter_Name": counter, "Counter_Value": value})


def test_traffic_scales_each_counter_by_the_copy_kernel(tmp_path):
    # a 1 MiB copy reads 512 KiB by FETCH_SIZE (scale 2) and 1024 KiB by
    # WRITE_SIZE (scale 1); the kernel's two dispatches (grid 640) read 100 and
    # 300 KiB (two counter instances each) and write 40 KiB; a dispatch of
    # another grid size is not the kernel's
    copy = "__amd_rocclr_copyBuffer"
    fetch = [(1, copy, 4096, "FETCH_SIZE", 512), (2, "k_force_wave<float>", 640, "FETCH_SIZE", 60),
             (2, "k_force_wave<float>", 640, "FETCH_SIZE", 40), (3, "k_force_wave<float>", 640, "FETCH_SIZE", 300),
             (4, "k_force_wave<float>", 128, "FETCH_SIZE", 9999)]
    write = [(1, copy, 4096, "WRITE_SIZE", 1024), (2, "k_force_wave<float>", 640, "WRITE_SIZE", 40),
             (3, "k_force_wave<float>", 640, "WRITE_SIZE", 40)]
    pf, pw = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _counters(pf, fetch)
    _counters(pw, write)
    r = profsum.traffic(str(pf), str(pw), "k_force_wave<float>", 640, 1024.0 * 1024.0)
    assert r["fetch_dispatches"] == 2 and r["fetch_kib_per_launch"] == 200.0
    assert r["fetch_scale"] == 2.0 and r["write_scale"] == 1.0
    assert r["traffic_bytes_per_launch"] == 1024.0 * (200.0 * 2.0 + 40.0 * 1.0)


def test_mix_averages_each_counter_per_dispatch_over_runs(tmp_path):
    # two counter runs of the same kernel: run a has two dispatches (the
    # counter reported in two instances for the first), run b one dispatch
    a = [(1, "k_force_wave<float>", 640, "SQ_INSTS_VALU", 70), (1, "k_force_wave<float>", 640, "SQ_INSTS_VALU", 30),
         (2, "k_force_wave<float>", 640, "SQ_INSTS_VALU", 300), (3, "k_build", 640, "SQ_INSTS_VALU", 5)]
    b = [(1, "k_force_wave<float>", 640, "SQ_INSTS_LDS", 12), (2, "k_force_wave<float>", 128, "SQ_INSTS_LDS", 99)]
    pa, pb = tmp_path / "a.csv", tmp_path / "b.csv"
    _counters(pa, a)
    _counters(pb, b)
    r, counts = profsum.mix([str(pa), str(pb)], "k_force_wave<float>", 640)
    assert r == {"SQ_INSTS_VALU": 200.0, "SQ_INSTS_LDS": 12.0}
    assert counts == {"SQ_INSTS_VALU": 2, "SQ_INSTS_LDS": 1}
