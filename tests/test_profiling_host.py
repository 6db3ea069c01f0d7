"""CPU tests of the profile summarizer (counter calibration, per-kernel rows, the
kernel-source digest) on small synthetic rocprofv3 CSV outputs."""

import csv
import os

from paper_2007_06524_amd import profiling as pf


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_summary_round_trip(tmp_path):
    trace = tmp_path / "trace"
    _write(str(trace / "t_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", 0, 90000],
            ["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", 100000, 190000],
            ["void k_gemm_16<1, 64, 64, 64, false, true, unsigned short>(GemmArgs)", 0, 50000],
            ["void at::native::vectorized_elementwise_kernel<4>", 0, 1000]])
    copy = "void at::native::vectorized_elementwise_kernel<4>"
    fetch = tmp_path / "fetch"
    # FETCH_SIZE reports half of the copy's 256 MiB read: factor 2.
    _write(str(fetch / "f_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[copy, "FETCH_SIZE", 128 * 1024],
            ["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", "FETCH_SIZE", 1000.0],
            ["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", "FETCH_SIZE", 3000.0],
            ["void k_gemm_16<1, 64, 64, 64, false, true, unsigned short>(GemmArgs)", "FETCH_SIZE", 7.0]])
    write = tmp_path / "write"
    _write(str(write / "w_counter_collection.csv"), ["Kernel_Name", "Counter_Name", "Counter_Value"],
           [[copy, "WRITE_SIZE", 256 * 1024],
            ["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", "WRITE_SIZE", 500.0],
            ["void k_gemm_16c<1, 128, 128, 64, false, unsigned short>(GemmArgs)", "WRITE_SIZE", 500.0]])
    text = pf.summarize(str(trace), str(fetch), str(write), 256, "t", ("cmd",), digest="abc")
    assert "FETCH_SIZE x 2.000, WRITE_SIZE x 1.000" in text
    out = tmp_path / "s.md"
    out.write_text(text)
    tr = pf.measured_traffic(str(out), r"k_gemm_16c?<1,")
    # the row with the most launches; average counter x factor, KiB -> bytes
    assert tr["launches"] == 2 and tr["digest"] == "abc"
    assert abs(tr["fetch_bytes"] - 2000.0 * 2 * 1024) < 0.5e6 * 0.1 + 1e3
    assert abs(tr["write_bytes"] - 500.0 * 1024) < 0.5e5
    assert pf.measured_traffic(str(out), r"no such kernel") is None


def test_digest_tracks_the_kernel_sources(tmp_path):
    csrc = tmp_path / "csrc"
    csrc.mkdir()
    (csrc / "a.hip").write_text("x")
    (csrc / "b.h").write_text("y")
    (csrc / "c.cpp").write_text("host only")
    d1 = pf.kernel_source_digest(str(tmp_path))
    (csrc / "c.cpp").write_text("changed host code")
    assert pf.kernel_source_digest(str(tmp_path)) == d1
    (csrc / "a.hip").write_text("x2")
    assert pf.kernel_source_digest(str(tmp_path)) != d1
    assert len(pf.kernel_source_digest()) == 64


def test_bench_rooflines_from_event_times():
    """bench.py's per-class rates: a GEMM stage is 2 R N^4 flop, and in 16-bit
    precision also (2 + 2R), 4R and 2R + 12 bytes per unknown for the three
    stages (16-bit input and intermediates of R N^3 values, the float z and the
    float r, q its dot products read); the stencil 2 words per unknown plus the
    L^3 cells; the FP64 residual reads x, f and writes one word.  Hand-computed
    numbers at N = 256, R = 5, 1 ms per launch."""
    import bench

    N, R, L = 256, 5, 64
    n3 = N ** 3
    timing = {"gemm_mode3": (2.0, 2), "gemm_mode2": (1.0, 1), "gemm_mode1": (3.0, 3),
              "stencil": (1.0, 1), "residual": (1.0, 1), "vector": (0.0, 0)}
    k = bench.kernel_rooflines(timing, N, R, "mixed_fp16", L)
    assert "vector" not in k                                   # no launches, no entry
    for name, per in (("gemm_mode3", 12), ("gemm_mode2", 20), ("gemm_mode1", 22)):
        g = k[name]
        assert g["avg_ms"] == 1.0 and g["bound"] == "mfma"
        assert abs(g["achieved"] - 2 * R * N ** 4 / 1e-3 / 1e12) < 1e-9 * g["achieved"]
        assert abs(g["frac"] - g["achieved"] / 2500.0) < 1e-15
        assert g["hbm"]["algorithmic"] == per * n3
        assert abs(g["hbm"]["achieved"] - per * n3 / 1e-3 / 1e9) < 1e-9 * g["hbm"]["achieved"]
        assert abs(g["hbm"]["flop_per_byte"] - 2 * R * N / per) < 1e-12
    assert k["stencil"]["algorithmic"] == 2 * 4 * n3 + 4 * L ** 3
    assert k["residual"]["algorithmic"] == (2 * 8 + 4) * n3
    k64 = bench.kernel_rooflines(timing, N, R, "fp64", L)
    assert "hbm" not in k64["gemm_mode1"] and k64["gemm_mode1"]["peak"] == 78.6
    assert k64["stencil"]["algorithmic"] == 2 * 8 * n3 + 8 * L ** 3
