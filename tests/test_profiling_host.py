"""The rocprofv3 summary tools on synthetic result databases (no GPU): kernel
durations, the copy-calibrated traffic and the kernel-name patterns."""
import json
import sqlite3

import pytest

from paper_1612_04040_amd import profiling as P

KIB = 1024.0


def _db(path, kernels=(), counters=()):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                "counter_name text, value real)")
    con.executemany("insert into kernels values (?, ?, ?)", kernels)
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    con.commit()
    con.close()
    return str(path)


def _pmc(path, counter, per_kernel, calib_kib):
    rows, d = [], 0
    for name, vals in per_kernel:
        for v in vals:
            rows.append((d, name, counter, v))
            d += 1
    for v in calib_kib:  # the calibration copies come last
        rows.append((d, "void ls::copy_f32_kernel(float*, float const*, long)", counter, v))
        d += 1
    return _db(path, counters=rows)


def test_kernel_durations_group_by_name_without_arguments(tmp_path):
    db = _db(tmp_path / "t.db", kernels=[
        ("void ls::brick_step2_kernel<float, 0>(ls::StepGeom, ls::StepArgs<float, float>)", 0, 40000),
        ("void ls::brick_step2_kernel<float, 0>(ls::StepGeom, ls::StepArgs<float, float>)", 50000, 70000),
        ("ls::item_record_kernel(ls::ItemRecordFn, int const*)", 0, 5000)])
    d = P.kernel_durations(db)
    assert d["ls::brick_step2_kernel<float, 0>"] == (2, 30.0)
    assert d["ls::item_record_kernel"] == (1, 5.0)


def test_traffic_scales_by_the_copy_and_matches_a_pattern(tmp_path):
    """FETCH_SIZE reads half of a dword copy's bytes (scale 2), WRITE_SIZE all
    of them (scale 1); the kernel pattern is a regular expression matched at
    the start of the name, so the reinitialisation kernels (modes 2 and 3)
    are taken and the cut-off ones (mode 1) are not."""
    gib_kib = (1 << 30) / KIB
    kern = [("ls::brick_step2_kernel<float, 2>", [100.0, 300.0]),   # mean 200 KiB
            ("ls::brick_step_kernel<float, 3>", [200.0]),
            ("ls::brick_step2_kernel<float, 1>", [9999.0])]
    f = _pmc(tmp_path / "f.db", "FETCH_SIZE", kern, [gib_kib / 2] * 3)
    w = _pmc(tmp_path / "w.db", "WRITE_SIZE", [(k, [v / 2 for v in vals]) for k, vals in kern],
             [gib_kib] * 3)
    rec = P.traffic(f, w, r"ls::brick_step2?_kernel<float, [23]>")
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["read_bytes"] == pytest.approx(2.0 * 200.0 * KIB)  # (100 + 300 + 200) / 3 KiB, x2
    assert rec["write_bytes"] == pytest.approx(100.0 * KIB)
    assert rec["dispatches"] == [3, 3]
    # a plain name prefix still works as a pattern
    assert P.traffic(f, w, "ls::brick_step2_kernel<float, 1>")["read_bytes"] == pytest.approx(
        2.0 * 9999.0 * KIB)


def test_traffic_cli_records_the_digest(tmp_path):
    gib_kib = (1 << 30) / KIB
    kern = [("ls::band_gather_chunk_kernel<float>", [50.0])]
    f = _pmc(tmp_path / "f.db", "FETCH_SIZE", kern, [gib_kib / 2] * 3)
    w = _pmc(tmp_path / "w.db", "WRITE_SIZE", kern, [gib_kib] * 3)
    out = tmp_path / "traffic.json"
    assert P.main(["traffic", f, w, "--kernel", "ls::band_gather", "--key", "gather/x",
                   "--digest", "abcd", "--out", str(out)]) == 0
    rec = json.loads(out.read_text())["gather/x"]
    assert rec["source_digest"] == "abcd"
    assert rec["kernels"] == ["ls::band_gather_chunk_kernel<float>"]
    assert P.main(["traffic", f, w, "--kernel", "ls::nothing", "--key", "k", "--digest", "d",
                   "--out", str(out)]) == 1
