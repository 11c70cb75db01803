"""The rocprofv3 summary tool on small synthetic result databases (CPU only)."""
import json
import sqlite3

import pytest

from paper_1908_06742_amd import profiling as P


def _kernels_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()


def _counters_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_kernel_stats_and_sequence(tmp_path, capsys):
    db = str(tmp_path / "t.db")
    rows, t = [], 0
    for it in range(4):                       # four iterations: conv 10 us, wgrad 20 us, adam 5 us, 1 us gaps
        for name, d in (("k_conv", 10_000), ("k_wgrad", 20_000), ("k_adam", 5_000)):
            rows.append((name, t, t + d))
            t += d + 1_000
    _kernels_db(db, rows)
    st = {k["name"]: k for k in P.kernel_stats(db)}
    assert st["k_wgrad"]["calls"] == 4 and st["k_wgrad"]["avg_ns"] == 20_000
    assert abs(sum(k["percent"] for k in st.values()) - 100.0) < 1e-9
    P.main(["sequence", db, "--marker", "k_adam"])
    out = capsys.readouterr().out.splitlines()
    # between the second and third adam: conv, wgrad, adam; busy 35 us; span = 3 gaps + 35 us
    assert out[-1] == "3 dispatches, kernel time 35.0 us, busy 35.0 us, span 38.0 us"
    with pytest.raises(SystemExit):
        P.main(["sequence", db, "--marker", "k_missing"])


def test_sequence_counts_overlapping_kernels_once(tmp_path, capsys):
    # per iteration: conv 0-10, wgrad 5-25 (second stream), sum 12-14 (inside wgrad),
    # adam 26-31; the next iteration starts at 40
    db = str(tmp_path / "o.db")
    rows = []
    for it in range(4):
        t = 40_000 * it
        rows += [("k_conv", t, t + 10_000), ("k_wgrad", t + 5_000, t + 25_000), ("k_sum", t + 12_000, t + 14_000),
                 ("k_adam", t + 26_000, t + 31_000)]
    _kernels_db(db, rows)
    P.main(["sequence", db, "--marker", "k_adam"])
    out = capsys.readouterr().out.splitlines()
    assert out[1].endswith("(overlaps 5.0 us)") and out[2].endswith("(overlaps 2.0 us)") and "overlaps" not in out[0]
    # kernel time 10 + 20 + 2 + 5 = 37; busy 0-25 and 26-31 = 30; span 31 - (-9) = 40
    assert out[-1] == "4 dispatches, kernel time 37.0 us, busy 30.0 us, span 40.0 us"


def test_counters_scale_by_the_copy_calibration(tmp_path, capsys):
    f, w, cf, cw = (str(tmp_path / n) for n in ("f.db", "w.db", "cf.db", "cw.db"))
    # the copy of 1 GiB reads FETCH_SIZE = 2^19 KiB (half) and writes WRITE_SIZE = 2^20 KiB:
    # fetch is scaled by 2, write by 1
    _counters_db(cf, [(1, "copyBuffer", "FETCH_SIZE", 2.0 ** 19)])
    _counters_db(cw, [(1, "copyBuffer", "WRITE_SIZE", 2.0 ** 20)])
    _counters_db(f, [(1, "k_step<even>", "FETCH_SIZE", 1000.0), (2, "k_step<even>", "FETCH_SIZE", 1000.0),
                     (3, "k_step<odd>", "FETCH_SIZE", 1100.0), (4, "other", "FETCH_SIZE", 9.0)])
    _counters_db(w, [(1, "k_step<even>", "WRITE_SIZE", 2000.0), (2, "k_step<even>", "WRITE_SIZE", 2000.0),
                     (3, "k_step<odd>", "WRITE_SIZE", 2000.0)])
    out = str(tmp_path / "c.json")
    P.main(["counters", f, w, cf, cw, "--kernel", "k_step", "--nodes", "100", "--bytes-per-node", "40",
            "--tile-width", "64", "--out", out])
    d = json.load(open(out))
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    per = {r["kernel"]: r for r in d["per_parity"]}
    assert per["k_step<even>"]["fetch_bytes"] == 2000.0 * 1024 and per["k_step<even>"]["write_bytes"] == 2000.0 * 1024
    assert per["k_step<odd>"]["fetch_bytes"] == 2200.0 * 1024
    assert d["bytes_per_launch"] == ((2000.0 + 2000.0) + (2200.0 + 2000.0)) * 1024 / 2
    assert d["algorithmic_bytes_per_launch"] == 4000 and "kernel_hash" in d


def test_mangled_names_left_by_the_profiler_are_shortened():
    assert P.readable("_ZN12_GLOBAL__N_110k_up2_bwd8EPKDF16bNS_7RowGridEiiiiiPDF16b") == \
        "(anonymous namespace)::k_up2_bwd8(...)"
    assert P.readable("_ZN3ddf6k_stepIfLi0EEEvPT_") == "ddf::k_step(...)"
    assert P.readable("void ddf::k_step<float>(float*)") == "void ddf::k_step<float>(float*)"
