"""The profile summariser on small synthetic rocprofv3 outputs (no GPU): the
copy-calibrated traffic per launch, the per-kernel counter medians, and the
kernel-trace averages that leave out the no-op launches."""
import csv

from paper_1103_1363_amd import prof_summary as ps

HDR = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        w.writerows(rows)


def test_traffic_is_copy_calibrated(tmp_path):
    # the reference copy moves 1 GiB each way; its counters read 2x (fetch)
    # and 1x (write) that in KiB, summed over two instances per dispatch
    gib_kib = (1 << 30) / 1024
    fetch = [(1, "stream_copy_kernel(...)", "FETCH_SIZE", gib_kib), (1, "stream_copy_kernel(...)", "FETCH_SIZE", gib_kib),
             (2, "void lq::cg_k4<lq::P16, lq::P32>(...)", "FETCH_SIZE", 1000.0),
             (2, "void lq::cg_k4<lq::P16, lq::P32>(...)", "FETCH_SIZE", 1000.0)]
    write = [(1, "stream_copy_kernel(...)", "WRITE_SIZE", gib_kib),
             (2, "void lq::cg_k4<lq::P16, lq::P32>(...)", "WRITE_SIZE", 500.0)]
    write_counters(tmp_path / "f.csv", fetch)
    write_counters(tmp_path / "w.csv", write)
    cf, cw, rows = ps.pmc_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"))
    assert abs(cf - 0.5) < 1e-12 and abs(cw - 1.0) < 1e-12
    got = {name: (f, w) for name, n, f, w in rows}
    f, w = got["cg_k4<P16, P32>"]
    assert abs(f - 2000.0 * 1024 * 0.5) < 1e-6
    assert abs(w - 500.0 * 1024) < 1e-6


def test_counter_table_takes_the_median_per_dispatch(tmp_path):
    rows = []
    for d, v in [(1, 10.0), (2, 30.0), (3, 20.0)]:
        rows.append((d, "void lq::dslash_kernel<lq::P16, false>(...)", "TA_TA_BUSY_sum", v))
        rows.append((d, "void lq::dslash_kernel<lq::P16, false>(...)", "SQ_WAVES", 4.0))
    rows.append((4, "other_kernel(...)", "SQ_WAVES", 1.0))
    write_counters(tmp_path / "c.csv", rows)
    tab = ps.counter_table([str(tmp_path / "c.csv")], match="^dslash")
    got = {(k, c): (n, v) for k, c, n, v in tab}
    assert got[("dslash_kernel<P16, false>", "TA_TA_BUSY_sum")] == (3, 20.0)
    assert got[("dslash_kernel<P16, false>", "SQ_WAVES")] == (3, 4.0)
    assert all(k.startswith("dslash") for k, _, _, _ in tab)


def test_trace_summary_drops_noop_launches(tmp_path):
    path = tmp_path / "t_kernel_trace.csv"
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for d in (100000, 100000, 100000, 1000):  # ns; the last is a no-op replay
            w.writerow(["void lq::cg_k1<lq::P16, false>(...)", 0, d])
    out = ps.summary(str(path))
    line = [ln for ln in out.splitlines() if ln.startswith("cg_k1")][0].split()
    calls, work_calls, work_avg = int(line[-6]), int(line[-3]), float(line[-2])
    assert calls == 4 and work_calls == 3 and abs(work_avg - 100.0) < 1e-9
