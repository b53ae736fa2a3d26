"""Summaries of rocprofv3 results (rocpd SQLite databases) as short text.

    python -m paper_2408_06698_amd.rocpd_summary trace <db> [top]
        per kernel name: launches, average / busy-average / max / total duration
    python -m paper_2408_06698_amd.rocpd_summary ranges <db>
        the library's roctx ranges (marker trace): calls, average / total time
    python -m paper_2408_06698_amd.rocpd_summary traffic <fetch_db> <write_db> <kernels.hip>
        HBM bytes per launch from a FETCH_SIZE and a WRITE_SIZE run, scaled by
        what the counters read for the largest plain device copy in the runs
"""
import hashlib
import re
import sqlite3
import statistics
import sys

# kernel keys of the traffic summary: substring of the demangled name
TRAFFIC_KERNELS = [
    ("mass_k3", "k_mass_lds<double, 3, 3, 0>"),
    ("prec_k3", "k_mass_lds<double, 3, 3, 1>"),
    ("elem_k3", "k_elem<double, 3, 3, 0>"),
    ("elem_fp32_k3", "k_elem<float, 3, 3, 0>"),
    ("modal_k3", "k_mass_lds<double, 3, 3, 2>"),
    ("mass_k5", "k_mass_tiled<double, 3, 5, 0>"),
    ("prec_k5", "k_mass_tiled<double, 3, 5, 1>"),
    ("elem_k5", "k_elem<double, 3, 5, 0>"),
    ("elem_fp32_k5", "k_elem<float, 3, 5, 0>"),
    ("modal_k5", "k_modal<double, 3, 5>"),
    ("rupdate", "k_rupdate<2>("),
    ("stokes_gemv", "k_stokes_gemv<9, double>"),
    ("xpay", "k_xpay<2>("),
    ("proj_k3", "k_proj<3, 3, 0>"),
]


def trace(db, top=20):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), sum(duration), min(duration), max(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    tot = sum(r[3] for r in rows)
    print("busy = launches longer than 5% of the kernel's longest (PCG launches queued after")
    print("convergence return at once; the library's own event timing leaves them out too)")
    print(f"{'launches':>8} {'avg_us':>10} {'busy_n':>7} {'busy_avg_us':>11} {'max_us':>9} {'total_ms':>9} {'pct':>6}  kernel")
    for r in rows[:top]:
        busy = c.execute("select count(*), avg(duration) from kernels where name = ? and duration > 0.05 * ?",
                         (r[0], r[5])).fetchone()
        print(f"{r[1]:8d} {r[2]/1e3:10.2f} {busy[0]:7d} {busy[1]/1e3:11.2f} {r[5]/1e3:9.2f} {r[3]/1e6:9.3f} "
              f"{100*r[3]/tot:6.2f}  {r[0][:110]}")


def ranges(db):
    """The library's roctx ranges (one per entry point call, and one per
    substep inside hopu_substeps): count, average and total host duration
    per range name, from a --marker-trace run."""
    c = sqlite3.connect(db)
    rows = c.execute("select json_extract(extdata, '$.message') as msg, count(*), avg(duration), sum(duration) "
                     "from regions where category like 'MARKER%' group by msg order by sum(duration) desc").fetchall()
    print("host time between the range's push and pop (the entry point's launches, its host work and, for")
    print("calls that synchronise, the wait for the GPU)")
    print(f"{'calls':>6} {'avg_ms':>10} {'total_ms':>10}  range")
    for msg, n, avg, tot in rows:
        print(f"{n:6d} {avg / 1e6:10.3f} {tot / 1e6:10.3f}  {msg}")


def _counter(db, name):
    """({kernel name: [per-dispatch values]}, value of the last dispatch) of
    one counter (KiB)."""
    c = sqlite3.connect(db)
    out = {}
    last = None
    for k, v in c.execute("select kernel_name, value from counters_collection where counter_name = ? "
                          "order by dispatch_id", (name,)):
        out.setdefault(k, []).append(float(v))
        last = (k, float(v))
    return out, last


def source_sha(text):
    """SHA-256 (16 hex) of a kernel source as the traffic summaries record
    it: for kernels.hip the part from 'namespace hopu {' to the launchers
    marker; for other sources the code with its // comments and blank lines
    removed (a comment edit does not change what the counters measured)."""
    marker = "// " + "-" * 66 + " launchers"
    if marker in text:
        text = text[text.index("namespace hopu {"):text.index(marker)]
    else:
        text = re.sub(r"//[^\n]*", "", text)
        text = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def kernels_sha(src):
    return source_sha(open(src).read())


def traffic(fetch_db, write_db, src):
    (fetch, flast), (write, wlast) = _counter(fetch_db, "FETCH_SIZE"), _counter(write_db, "WRITE_SIZE")
    # calibration: the last dispatch of each run, the 1 GiB device-to-device
    # copy that bench.py --copy-calib makes after everything else
    copy_bytes = 1 << 30
    assert "copy" in flast[0].lower() and "copy" in wlast[0].lower(), (flast[0], wlast[0])
    fmax, wmax = flast[1], wlast[1]
    fs, ws = copy_bytes / (fmax * 1024), copy_bytes / (wmax * 1024)
    print(f"# calibration: 1 GiB device copy ({flast[0]}) reads back FETCH_SIZE {fmax:.1f} KiB, "
          f"WRITE_SIZE {wmax:.1f} KiB")
    print(f"#   -> fetch scale {fs:.4f}, write scale {ws:.4f} (bytes = KiB * 1024 * scale)")
    print(f"# kernels_sha: SHA-256 (16 hex) of {src.split('/')[-1]} (kernels.hip: from 'namespace hopu {{' "
          "to the launchers marker; other sources without // comments and blank lines)")
    print("# per-launch medians over the launches at full size (> 80% of the kernel's largest)")
    print(f"kernels_sha = {kernels_sha(src)}")
    print(f"fetch_scale = {fs:.6f}")
    print(f"write_scale = {ws:.6f}")
    for key, pat in TRAFFIC_KERNELS:
        fk = [k for k in fetch if pat in k]
        wk = [k for k in write if pat in k]
        if not fk or not wk:
            continue
        fv = [x for x in fetch[fk[0]] if x > 0.8 * max(fetch[fk[0]])]
        wv = [x for x in write[wk[0]] if x > 0.8 * max(write[wk[0]])]
        f, w = statistics.median(fv), statistics.median(wv)
        print(f"# {key}: FETCH_SIZE {f:.0f} KiB (n={len(fv)}), WRITE_SIZE {w:.0f} KiB (n={len(wv)})")
        print(f"{key}_bytes_per_launch = {f * 1024 * fs + w * 1024 * ws:.0f}")


BUSY_KERNELS = TRAFFIC_KERNELS + [("elem_bf16x2_k3", "k_elem<float, 3, 3, 2>"),
                                  ("elem_bf16x3_k3", "k_elem<float, 3, 3, 3>"),
                                  ("prec_fp32_k3", "k_mass_lds<float, 3, 3, 1>"),
                                  ("elem_bf16x2_k5", "k_elem<float, 3, 5, 2>"),
                                  ("elem_bf16x3_k5", "k_elem<float, 3, 5, 3>"),
                                  ("prec_fp32_k5", "k_mass_tiled<float, 3, 5, 1>"),
                                  ("stokes_gemv_fp32", "k_stokes_gemv<9, float>"),
                                  ("stokes_setup", "k_stokes_setup(")]
N_SIMD = 256 * 4  # MI355X: 256 CUs, 4 SIMDs each
N_XCD = 8


def busy(db):
    """MFMA and VALU utilisation per kernel from one counter run.  The SQ
    counters are summed over the chip's 1024 SIMDs; GRBM_GUI_ACTIVE reads the
    sum over the 8 XCDs, so the dispatch's cycles are GRBM_GUI_ACTIVE / 8
    (at 2.4 GHz that matches the launch durations).  SQ_WAVE_CYCLES and
    SQ_ACTIVE_INST_VALU count quad-cycles, SQ_VALU_MFMA_BUSY_CYCLES cycles.
    Per-launch medians over the launches at full size."""
    names = ["GRBM_GUI_ACTIVE", "SQ_VALU_MFMA_BUSY_CYCLES", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES",
             "SQ_WAVE_CYCLES"]
    vals = {n: _counter(db, n)[0] for n in names}
    print("# cycles     = GRBM_GUI_ACTIVE / 8 XCDs")
    print("# MFMA busy  = SQ_VALU_MFMA_BUSY_CYCLES / (cycles * 1024 SIMDs)")
    print("# VALU busy  = 4 * SQ_ACTIVE_INST_VALU / (cycles * 1024 SIMDs)")
    print("# waves/SIMD = 4 * SQ_WAVE_CYCLES / (cycles * 1024 SIMDs)  (mean resident waves)")
    print("# per-launch medians over the launches at full size (GRBM_GUI_ACTIVE > 80% of the kernel's largest)")
    print(f"{'key':<12} {'n':>4} {'cycles':>9} {'us@2.4GHz':>9} {'mfma_busy':>9} {'valu_busy':>9} {'waves/simd':>10}  kernel")
    for key, pat in BUSY_KERNELS:
        ks = [k for k in vals["GRBM_GUI_ACTIVE"] if pat in k]
        if not ks:
            continue
        k = ks[0]
        g = vals["GRBM_GUI_ACTIVE"][k]
        keep = [i for i, x in enumerate(g) if x > 0.8 * max(g)]
        med = {n: statistics.median([vals[n][k][i] for i in keep]) for n in names}
        cyc = med["GRBM_GUI_ACTIVE"] / N_XCD
        den = cyc * N_SIMD
        print(f"{key:<12} {len(keep):4d} {cyc:9.0f} {cyc / 2400:9.1f} {med['SQ_VALU_MFMA_BUSY_CYCLES'] / den:9.3f} "
              f"{4 * med['SQ_ACTIVE_INST_VALU'] / den:9.3f} {4 * med['SQ_WAVE_CYCLES'] / den:10.2f}  {k[:64]}")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 20)
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "busy":
        busy(sys.argv[2])
    elif sys.argv[1] == "ranges":
        ranges(sys.argv[2])
    else:
        trace(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 20)
