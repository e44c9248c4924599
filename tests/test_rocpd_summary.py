"""The rocprofv3 database summaries (host only): a synthetic database with
the two views the summaries read."""
import sqlite3

from paper_1905_01381_amd import rocpd_summary as rs


def _db(path, kernels, pmc):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, duration integer)")
    c.execute("create table pmc_events (dispatch_id integer, name text, duration integer, counter_name text, "
              "counter_value real)")
    c.executemany("insert into kernels values (?, ?)", kernels)
    c.executemany("insert into pmc_events values (?, ?, ?, ?, ?)", pmc)
    c.commit()
    c.close()
    return str(path)


def test_trace_table(tmp_path):
    db = _db(tmp_path / "t.db", [("eri_jk_dddp(PairSet, ...)", 2_000_000), ("eri_jk_dddp(PairSet, ...)", 4_000_000),
                                 ("fill_kernel(double*)", 1_000_000)], [])
    out = rs.trace(db)
    assert "| eri_jk_dddp | 2 | 6.00 | 3.000 | 2.000 | 4.000 | 85.7 |" in out
    assert "| fill_kernel | 1 | 1.00 |" in out


def test_traffic_calibrated_by_copy(tmp_path):
    # a 1 MiB copy reads 512 KiB of FETCH_SIZE (factor 2) and writes 1024 KiB (factor 1)
    f = _db(tmp_path / "f.db", [], [(1, "__amd_rocclr_copyBuffer", 1000, "FETCH_SIZE", 256.0),
                                    (1, "__amd_rocclr_copyBuffer", 1000, "FETCH_SIZE", 256.0),
                                    (2, "eri_jk_ssss(...)", 1_000_000, "FETCH_SIZE", 1000.0)])
    w = _db(tmp_path / "w.db", [], [(1, "__amd_rocclr_copyBuffer", 1000, "WRITE_SIZE", 1024.0),
                                    (2, "eri_jk_ssss(...)", 1_000_000, "WRITE_SIZE", 500.0)])
    out = rs.traffic(f, w, 1.0)
    assert "factor 2.0000" in out and "factor 1.0000" in out
    # 1000 KiB x 2 x 1024 B = 2.048 MB read; 500 KiB x 1024 B = 0.512 MB written
    row = [l for l in out.splitlines() if l.startswith("| eri_jk_ssss")][0]
    assert "| 0.00 | 0.00 |" in row and "| 1.00 |" in row


def test_valu_rates(tmp_path):
    # 1 ms, 2.4e6 cycles; 1024 SIMDs x 2.4e6 x 0.25 = 6.144e8 slots, half used
    db = _db(tmp_path / "s.db", [], [(1, "eri_jk_pppp(...)", 1_000_000, "SQ_INSTS_VALU", 3.072e8),
                                     (1, "eri_jk_pppp(...)", 1_000_000, "SQ_INSTS_VALU_FLOPS_FP64", 1e9),
                                     (1, "eri_jk_pppp(...)", 1_000_000, "GRBM_GUI_ACTIVE", 2.4e6),
                                     (1, "eri_jk_pppp(...)", 1_000_000, "GRBM_GUI_ACTIVE", 2.4e6),
                                     (1, "eri_jk_pppp(...)", 1_000_000, "SQ_WAVES", 64)])
    row = [l for l in rs.valu(db).splitlines() if l.startswith("| eri_jk_pppp")][0]
    assert "| 6.400e+10 | 64.0 | 0.50 | 64 |" in row
