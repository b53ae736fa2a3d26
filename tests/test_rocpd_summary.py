"""Host logic of the rocprofv3 summaries (paper_2408_06698_amd.rocpd_summary)
on small synthetic result databases: busy filtering of the trace, the copy
calibration of the HBM counters and the utilisation arithmetic."""
import sqlite3

import pytest

from paper_2408_06698_amd import rocpd_summary as R

MASS = "void hopu::k_mass_lds<double, 3, 3, 0>(double const*)"
ELEM = "void hopu::k_elem<double, 3, 3, 0>(double const*)"
COPY = "__amd_rocclr_copyBuffer"


def _kernels_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, duration integer)")
    c.executemany("insert into kernels values (?, ?)", rows)
    c.commit()
    c.close()


def _counters_db(path, rows):
    """rows: (dispatch_id, kernel_name, counter_name, value)"""
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
              "value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()


def test_trace_busy_average_skips_short_launches(tmp_path, capsys):
    db = str(tmp_path / "t.db")
    # three full launches of 80 us and two that returned at once (1 us)
    _kernels_db(db, [(MASS, 80_000)] * 3 + [(MASS, 1_000)] * 2 + [(ELEM, 500_000)])
    R.trace(db)
    out = capsys.readouterr().out.splitlines()
    row = [l for l in out if "k_mass_lds" in l][0].split()
    launches, avg, busy_n, busy_avg = int(row[0]), float(row[1]), int(row[2]), float(row[3])
    assert launches == 5 and busy_n == 3
    assert avg == pytest.approx((3 * 80 + 2 * 1) / 5)
    assert busy_avg == pytest.approx(80.0)
    # ordered by total time: the element kernel (500 us) comes first
    assert out.index([l for l in out if "k_elem" in l][0]) < out.index([l for l in out if "k_mass_lds" in l][0])


def test_traffic_scales_by_the_copy_calibration(tmp_path, capsys):
    src = tmp_path / "kernels.hip"
    src.write_text("// head\nnamespace hopu {\nint body;\n// " + "-" * 66 + " launchers\nint tail;\n")
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    gib_kib = (1 << 30) / 1024
    # the counters read half the copy's true bytes (scale 2) on fetch and
    # exactly its bytes on write (scale 1); one short mass dispatch is left
    # out by the 80% filter
    _counters_db(fdb, [(1, MASS, "FETCH_SIZE", 1000.0), (2, MASS, "FETCH_SIZE", 1000.0),
                       (3, MASS, "FETCH_SIZE", 10.0), (4, COPY, "FETCH_SIZE", gib_kib / 2)])
    _counters_db(wdb, [(1, MASS, "WRITE_SIZE", 300.0), (2, MASS, "WRITE_SIZE", 300.0),
                       (3, COPY, "WRITE_SIZE", gib_kib)])
    R.traffic(fdb, wdb, str(src))
    vals = {}
    for line in capsys.readouterr().out.splitlines():
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            vals[a.strip()] = b.strip()
    assert float(vals["fetch_scale"]) == pytest.approx(2.0)
    assert float(vals["write_scale"]) == pytest.approx(1.0)
    assert float(vals["mass_k3_bytes_per_launch"]) == pytest.approx(1000 * 1024 * 2 + 300 * 1024)
    assert vals["kernels_sha"] == R.kernels_sha(str(src)) and len(vals["kernels_sha"]) == 16
    assert "elem_k3_bytes_per_launch" not in vals


def test_traffic_requires_the_copy_last(tmp_path):
    src = tmp_path / "kernels.hip"
    src.write_text("namespace hopu {\n// " + "-" * 66 + " launchers\n")
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _counters_db(fdb, [(1, MASS, "FETCH_SIZE", 1000.0)])
    _counters_db(wdb, [(1, MASS, "WRITE_SIZE", 300.0)])
    with pytest.raises(AssertionError):
        R.traffic(fdb, wdb, str(src))


def test_busy_utilisation_arithmetic(tmp_path, capsys):
    db = str(tmp_path / "b.db")
    cyc = 100_000  # per-XCD cycles of the dispatch
    simd = R.N_SIMD
    vals = {"GRBM_GUI_ACTIVE": cyc * R.N_XCD,
            "SQ_VALU_MFMA_BUSY_CYCLES": 0.5 * cyc * simd,  # half the SIMD cycles
            "SQ_ACTIVE_INST_VALU": 0.25 * cyc * simd / 4,   # quad-cycles: a quarter busy
            "SQ_BUSY_CYCLES": cyc,
            "SQ_WAVE_CYCLES": 2.0 * cyc * simd / 4}         # two resident waves per SIMD
    _counters_db(db, [(1, MASS, n, v) for n, v in vals.items()])
    R.busy(db)
    row = [l for l in capsys.readouterr().out.splitlines() if l.startswith("mass_k3 ")][0].split()
    assert int(row[1]) == 1
    assert float(row[2]) == pytest.approx(cyc)
    assert float(row[3]) == pytest.approx(cyc / 2400, abs=0.05)
    assert float(row[4]) == pytest.approx(0.5)
    assert float(row[5]) == pytest.approx(0.25)
    assert float(row[6]) == pytest.approx(2.0)


def test_ranges_grouped_by_message(tmp_path, capsys):
    db = str(tmp_path / "r.db")
    c = sqlite3.connect(db)
    c.execute("create table regions (category text, extdata text, duration integer)")
    rows = [("MARKER_CORE_RANGE_API", '{"message":"substep"}', 10_000_000)] * 3 + \
           [("MARKER_CORE_RANGE_API", '{"message":"hopu_substeps"}', 31_000_000),
            ("HIP_RUNTIME_API", '{"message":"ignored"}', 5)]
    c.executemany("insert into regions values (?, ?, ?)", rows)
    c.commit()
    c.close()
    R.ranges(db)
    out = capsys.readouterr().out.splitlines()
    sub = [l for l in out if l.endswith(" substep")][0].split()
    assert int(sub[0]) == 3 and float(sub[1]) == pytest.approx(10.0) and float(sub[2]) == pytest.approx(30.0)
    assert not any("ignored" in l for l in out)
    # ordered by total time: hopu_substeps (31 ms) before substep (30 ms)
    assert out.index([l for l in out if l.endswith("hopu_substeps")][0]) < out.index([l for l in out if l.endswith(" substep")][0])
