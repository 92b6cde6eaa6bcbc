"""The rocprofv3 CSV summariser on small synthetic CSV files (CPU only)."""
import csv
import hashlib
import json
import os

from paper_1108_5882_amd import profile_summary as ps


def _write(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_trace_and_traffic(tmp_path):
    d = tmp_path / "trace"
    d.mkdir()
    hdr = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    _write(d / "x_kernel_trace.csv", hdr, [["K", 1, "nll_stream_kernel<a>", 0, 120000],
                                           ["K", 2, "nll_stream_kernel<a>", 200000, 322000],
                                           ["K", 3, "other", 0, 5000],
                                           ["K", 4, "nll_stream_kernel<a>", 400000, 410000]])
    t = ps.trace_table(str(d), "nll_stream", min_us=100)
    assert t["nll_stream_kernel<a>"]["launches"] == 2
    assert abs(t["nll_stream_kernel<a>"]["mean"] - 121.0) < 1e-9
    fdir, wdir = tmp_path / "f", tmp_path / "w"
    fdir.mkdir()
    wdir.mkdir()
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the kernel: 3 dispatches, the last two counted; the copy of 1 MiB reads 2x its counter
    _write(fdir / "f_counter_collection.csv", hdr, [[1, "nll_stream_kernel<a>", "FETCH_SIZE", 999.0],
                                                     [2, "nll_stream_kernel<a>", "FETCH_SIZE", 500.0],
                                                     [3, "nll_stream_kernel<a>", "FETCH_SIZE", 502.0],
                                                     [4, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 512.0]])
    _write(wdir / "w_counter_collection.csv", hdr, [[2, "nll_stream_kernel<a>", "WRITE_SIZE", 1.0],
                                                     [3, "nll_stream_kernel<a>", "WRITE_SIZE", 3.0],
                                                     [4, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1024.0]])
    src, src2 = tmp_path / "src.hpp", tmp_path / "reduce.hpp"
    src.write_text("kernel")
    src2.write_text("combine")
    out = tmp_path / "traffic"
    ps.main(["traffic", str(fdir), str(wdir), "--kernel", "nll_stream", "--last", "2", "--copy-bytes",
             str(1 << 20), "--alg-bytes", str(1 << 20), "--units", "10", "--config", "cfg A", "--source", str(src),
             "--source", str(src2), "--command", "cmd", "--out", str(out)])
    rec = json.load(open(str(out) + ".json"))
    # the hash covers the source files concatenated in order, as the bench computes it
    assert rec["kernel_sha256_16"] == hashlib.sha256(b"kernelcombine").hexdigest()[:16]
    assert rec["kernel"] == "cfg A" and rec["units_per_launch"] == 10
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert abs(rec["hbm_bytes_per_launch"] - (501.0 * 1024 * 2 + 2.0 * 1024)) < 1e-6
    assert os.path.exists(str(out) + ".md")


def test_bench_hash_covers_the_kernel_sources():
    """The bench keys stored traffic on every file the streaming kernel's code comes from."""
    import bench
    names = [os.path.basename(p) for p in bench.KERNEL_SRCS]
    assert names == ["nll_stream_impl.hpp", "block_reduce.hpp"]
    h = hashlib.sha256()
    for p in bench.KERNEL_SRCS:
        h.update(open(p, "rb").read())
    assert bench.kernel_hash() == h.hexdigest()[:16]
