"""Host-side pieces of bench.py: the rocprofv3 database readers, on small
SQLite files laid out like rocprofv3's `kernels` and `counters_collection`
views."""
import os
import sqlite3
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

K = "void fftc::stockham_spec<fftc::SpecCfg<float, 4096, 256, 1, false, false>, 16, 16, 16>"


def test_headline_key():
    assert bench.headline_key(K + "(float2 const*)") == "c64_4096_fwd"
    assert bench.headline_key(K.replace("1, false, false", "1, true, false")) == "c64_4096_inv"
    assert bench.headline_key(K.replace(", false, false>", ", false>")) == "c64_4096_fwd"
    assert bench.headline_key("void fftc::split_fft<4096, 2, false>") is None
    assert bench.headline_key(K.replace("float,", "double,")) is None


def _dbs(tmp_path):
    tr = tmp_path / "trace.db"
    db = sqlite3.connect(tr)
    db.execute("create table kernels (name, grid_x, grid_y, grid_z, workgroup_x, workgroup_y, workgroup_z, "
               "duration, vgpr_count, accum_vgpr_count, lds_size, scratch_size)")
    for d in (40000, 60000):  # ns
        db.execute("insert into kernels values (?, 1048576, 1, 1, 256, 1, 1, ?, 64, 0, 33280, 0)", (K + "(x)", d))
    db.execute("insert into kernels values (?, 2048, 1, 1, 256, 1, 1, 1000, 64, 0, 33280, 0)", (K + "(x)",))
    db.commit()
    pm = tmp_path / "pmc.db"
    db = sqlite3.connect(pm)
    db.execute("create table counters_collection (kernel_name, grid_size, workgroup_size, counter_name, value)")
    vals = {"SQ_WAVES": 16384, "SQ_INSTS_LDS": 1000, "SQ_LDS_BANK_CONFLICT": 250, "SQ_WAIT_INST_LDS": 30,
            "SQ_WAVE_CYCLES": 300, "SQ_VALU_MFMA_BUSY_CYCLES": 1024 * 100, "GRBM_GUI_ACTIVE": 8 * 400,
            "TCC_EA0_RDREQ_128B": 2 ** 20, "TCC_EA0_RDREQ_64B": 0, "TCC_EA0_RDREQ_32B": 2 ** 10,
            "TCC_EA0_WRREQ": 2 ** 21 + 2 ** 10, "TCC_EA0_WRREQ_64B": 2 ** 21, "MeanOccupancyPerCU": 12.5}
    for cn, v in vals.items():
        db.execute("insert into counters_collection values (?, 1048576, 256, ?, ?)", (K + "(x)", cn, v))
    db.commit()
    return str(tr), str(pm)


def test_counter_report_derived_rates(tmp_path, capsys):
    tr, pm = _dbs(tmp_path)
    bench.counter_report(tr, [pm])
    out = capsys.readouterr().out.splitlines()
    row = [r for r in out if "| 1048576 |" in r][0].split("|")
    cells = [c.strip() for c in row[1:-1]]
    assert cells[3] == "2" and cells[4] == "50.00"       # two dispatches, mean 50 us
    assert cells[6] == "16384" and cells[8] == "%.1f" % (1000 / 16384)
    assert cells[10] == "0.25"                            # conflict cycles per LDS instruction
    assert cells[11] == "10.0%"                          # LDS wait share
    assert cells[12] == "25.0%"                          # 1024 * 100 / (400 * 1024)
    assert cells[13] == "12.5"
    rd, wr = 2 ** 27 + 2 ** 15, 2 ** 27 + 2 ** 15
    assert cells[14] == "%.1f / %.1f" % (rd / 2 ** 20, wr / 2 ** 20)
    assert cells[15] == "%.0f" % ((rd + wr) / 50e3)
    small = [r for r in out if "| 2048 |" in r][0]       # traced only: counters missing
    assert small.count("| - |") >= 5


def test_counter_report_needs_counter_run():
    import subprocess
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"),
                        "--counter-report", "only_trace.db"], capture_output=True, text=True)
    assert r.returncode != 0 and "counter run" in r.stderr


def test_split_mfma_busy_from_profile():
    """The precision study quotes the counters' MfmaUtil for its split-precision
    launches from the committed report, guarded by the split kernel's source
    hash recorded there."""
    busy = bench.split_mfma_busy()
    import re
    text = open(os.path.join(bench.ROOT, "profiles", "hot_path_counters.md")).read()
    m = re.search(r"split-kernel source hash: ([0-9a-f]{16})", text)
    if not m or m.group(1) != bench.file_hash(bench.SPLIT_SOURCES):
        assert busy == {}
        pytest.skip("the counter report predates the current split-kernel sources")
    assert set(busy) == {(n, mode) for n in (1024, 4096, 16384) for mode in bench.SPLIT_MODE_NUMBER}
    assert all(0.0 < v < 1.0 for v in busy.values())
    assert busy[(4096, "split3_bf16")] > busy[(4096, "f16")]  # twice the products per group
