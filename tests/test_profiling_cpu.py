"""Host logic of the profile summaries (no GPU): the HBM traffic of the warp
kernel from FETCH_SIZE / WRITE_SIZE scaled by the calibration copy, the
kernel-trace statistics, the machine-readable lines the bench reads back,
and the per-counter means of the wait-counter summary.  The rocprofv3
databases are stand-ins with the tables and columns the summaries read."""
from __future__ import annotations

import os
import sqlite3

import pytest

from paper_2506_15183_amd import profiling as P

WARP = "void yoro::(anonymous namespace)::warp_batch_kernel<9>(yoro::BatchHeader*, yoro::DevJob const*, int)"
COPY = "void at::native::vectorized_elementwise_kernel<4, at::native::bitwise_not_kernel_cuda>(int, ...)"


def _db(path, kernels=(), counters=()):
    os.makedirs(path, exist_ok=True)
    c = sqlite3.connect(os.path.join(path, "x_results.db"))
    c.execute("create table kernels (name text, duration real)")
    c.execute("create table counters_collection (kernel_name text, counter_name text, value real)")
    c.executemany("insert into kernels values (?, ?)", kernels)
    c.executemany("insert into counters_collection values (?, ?, ?)", counters)
    c.commit()
    c.close()


def test_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    out = str(tmp_path)
    # Trace: five warp launches (median 530 us) and a shorter kernel.
    _db(os.path.join(out, "trace"), kernels=[(WARP, d) for d in (540e3, 520e3, 530e3, 529e3, 600e3)]
        + [("upload_kernel", 2e3)] * 3)
    # The copy moves COPY_BYTES each way; FETCH reports half of it, WRITE all.
    copy_fetch_kib = P.COPY_BYTES / 2 / 1024
    copy_write_kib = P.COPY_BYTES / 1024
    _db(os.path.join(out, "fetch"), counters=[(WARP, "FETCH_SIZE", 1000.0), (WARP, "FETCH_SIZE", 1200.0),
                                              (COPY, "FETCH_SIZE", copy_fetch_kib)])
    _db(os.path.join(out, "write"), counters=[(WARP, "WRITE_SIZE", 700.0), (COPY, "WRITE_SIZE", copy_write_kib)])
    pixels = 1000
    text = P.summarize(out, pixels)
    fetch = 1100.0 * 1024 * 2.0  # mean of the warp dispatches, fetch scale 2
    write = 700.0 * 1024 * 1.0
    path = os.path.join(out, "summary.md")
    with open(path, "w") as f:
        f.write(text)
    traffic, sha = P.read_summary(path)
    assert traffic == round(fetch + write)
    assert sha == P.kernel_source_sha()
    assert "kernel_median_ns: 530000" in text
    assert f"measured / algorithmic: {(fetch + write) / (12 * pixels):.4f}" in text
    # The trace table lists the warp kernel first (largest total time).
    first_row = [ln for ln in text.splitlines() if ln.startswith("| `")][0]
    assert "warp_batch_kernel" in first_row and "| 5 |" in first_row


def test_missing_calibration_is_an_error(tmp_path):
    out = str(tmp_path)
    _db(os.path.join(out, "fetch"), counters=[(WARP, "FETCH_SIZE", 1000.0)])
    with pytest.raises(RuntimeError):
        P._counter_means(os.path.join(out, "fetch"), "FETCH_SIZE")
    with pytest.raises(FileNotFoundError):
        P._db(os.path.join(out, "nothing_here"))


def test_read_summary_of_a_missing_or_partial_file(tmp_path):
    assert P.read_summary(str(tmp_path / "absent.md")) == (None, None)
    p = tmp_path / "partial.md"
    p.write_text("kernel_source_sha: abc123\n")
    assert P.read_summary(str(p)) == (None, "abc123")


def test_counter_means_of_the_warp_kernel_only(tmp_path):
    out = str(tmp_path / "pmc")
    _db(out, counters=[(WARP, "SQ_WAIT_ANY", 10.0), (WARP, "SQ_WAIT_ANY", 30.0), (WARP, "SQ_WAVE_CYCLES", 80.0),
                       (COPY, "SQ_WAIT_ANY", 1e9)])
    lines = P.summarize_warp_counters(out).splitlines()
    assert lines[0] == f"kernel_source_sha: {P.kernel_source_sha()}"
    assert "SQ_WAIT_ANY: 20 (mean of 2 dispatches)" in lines
    assert "SQ_WAVE_CYCLES: 80 (mean of 1 dispatches)" in lines
