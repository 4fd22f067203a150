"""The rocprofv3 summariser on small synthetic csv files: kernel names to
step slots, copy-calibrated traffic, the last-dispatch averages and the
issue fractions."""
import csv
import json

from paper_2311_14140_amd import rocprof_summary as rs


def _write(path, header, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_names_map_to_step_slots():
    assert rs.short_name("void dsmc::(anonymous namespace)::k_move_scatter_wide<float, false>"
                         "(dsmc::InstDesc const*, HIP_vector_type<int, 2u> const*)") == \
        "k_move_scatter_wide<float, false>"
    cases = {"k_count<float, false>": "count", "k_colsum": "colsum", "k_scan": "scan",
             "k_scan_small": "scan", "k_scan_seg": "scan", "k_colprefix": "colprefix",
             "k_move_scatter<double, true>": "move_scatter",
             "k_move_scatter_wide<float, false>": "move_scatter",
             "k_collide_bucket<float>": "collide", "k_collide_fast<float, 8>": "collide",
             "k_collide_det": "collide", "k_resident<float, true>": "resident",
             "k_finalize": "finalize", "__amd_rocclr_copyBuffer": None, "k_scatter<float>": None}
    for name, slot in cases.items():
        assert rs.phase(name) == slot, name


def test_traffic_is_scaled_by_the_copy_and_recorded(tmp_path):
    stats = tmp_path / "s" / "x_kernel_stats.csv"
    _write(stats, ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"],
           [["k_collide_bucket<float>", 4, 400000, 100000, 80.0],
            ["__amd_rocclr_copyBuffer", 1, 50000, 50000, 20.0]])
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the copy of 256 MiB reads half of its bytes on the fetch counter
    _write(tmp_path / "f" / "x_counter_collection.csv", hdr,
           [[1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 128 * 1024],
            [2, "k_collide_bucket<float>", "FETCH_SIZE", 1000], [2, "k_collide_bucket<float>", "FETCH_SIZE", 500],
            [3, "k_collide_bucket<float>", "FETCH_SIZE", 1500]])
    _write(tmp_path / "w" / "x_counter_collection.csv", hdr,
           [[1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 256 * 1024],
            [2, "k_collide_bucket<float>", "WRITE_SIZE", 3000], [3, "k_collide_bucket<float>", "WRITE_SIZE", 1000]])
    out = tmp_path / "t.json"
    rs.main(["traffic", "--stats", str(tmp_path / "s"), "--fetch", str(tmp_path / "f"),
             "--write", str(tmp_path / "w"), "--tag", "T", "--workload", "W", "--json", str(out)])
    rec = json.load(open(out))["T"]
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    # per dispatch: fetch 1500 KiB (the two rows of dispatch 2 add up), write 2000 KiB
    assert rec["fetch_KiB"]["collide"] == 1500.0 and rec["write_KiB"]["collide"] == 2000.0
    assert rec["bytes_per_launch"]["collide"] == (1500.0 * 2 + 2000.0) * 1024
    assert rec["avg_us"]["collide"] == 100.0
    assert rec["kernel_source_hash"] == rs.source_hash()


def test_last_dispatches_average_the_tail(tmp_path):
    hdr = ["Kernel_Name", "Dispatch_Id", "Start_Timestamp", "End_Timestamp"]
    rows = [["k_count<float, false>", i, 1000 * i, 1000 * i + (900 if i < 6 else 300)] for i in range(1, 9)]
    rows += [["k_finalize", 20, 0, 5000], ["k_resident<float, false>", 21, 0, 9000]]
    _write(tmp_path / "k" / "x_kernel_trace.csv", hdr, rows)
    got = rs.last_dispatches(str(tmp_path / "k"), 3)
    assert got == [("k_count<float, false>", 3, 300.0)]


def test_source_hash_ignores_comments_only():
    a = 'int f(int x) { // add one\n  return x + 1; /* done */ }\nconst char* s = "a // b";'
    b = 'int f(int x) {\n    return x + 1;   }\n// another note\nconst char* s = "a // b";'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "a // b";'
    assert rs._code_only(a) == rs._code_only(b)
    assert rs._code_only(a) != rs._code_only(c)
    assert '"a // b"' in rs._code_only(a)
