"""Host-side helpers of bench.py: the kernel named for each pass, and the
parsing of the counter summaries (on a summary written here, with the
digest of the current sources)."""
import os

import pytest

import bench


@pytest.mark.parametrize("pas,N,prec,name", [
    ("yc", 128, "f32", "k_yc_p<float,128>"),
    ("yc", 256, "f32", "k_yc_p<float,256>"),
    ("yc", 256, "f64", "k_yc_r<double,256>"),
    ("zf", 256, "f32", "k_zf_r<float,256>"),
    ("yc", 96, "f32", "k_yc_p<float,96>"),
    ("zi", 96, "f32", "k_zi_p<float,96>"),
    ("yc", 96, "f64", "k_yc<double,96>"),
    ("xf", 128, "f32", "k_xf<float,128>"),
    ("zi", 32, "f64", "k_zi_p<double,32>"),
])
def test_kernel_names(pas, N, prec, name):
    assert bench.kernel_name(pas, N, prec) == name


def test_counter_summary_parsing(tmp_path, monkeypatch):
    f = tmp_path / "summary.txt"
    f.write_text("\n".join([
        "# comment",
        f"csrc_sha256 {bench.source_digest()}",
        "kernel k_yc_p<float,128>",
        "systems_per_dispatch 16",
        "dispatches 10",
        "fetch_kib_per_dispatch 1000.0",
        "write_kib_per_dispatch 2000.0",
        "copy_bytes 1048576",
        "copy_fetch_kib 512.0",
        "copy_write_kib 1024.0",
        "bq::k_yc_p<float, 128>: SQ_INSTS_VALU 2e+08, SQ_WAVES 2.6e+05",
    ]) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILES", (str(f),))
    t = bench.measured_traffic("k_yc_p<float,128>", 16)
    # fetch scaled by 1 MiB / 512 KiB = 2, write by 1
    assert t["fetch_bytes"] == 2 * 1000 * 1024 and t["write_bytes"] == 2000 * 1024
    assert bench.measured_traffic("k_yc_p<float,128>", 15) is None
    assert bench.measured_sq("k_yc_p<float,128>", 16)["SQ_INSTS_VALU"] == 2e8
    r = {"kernel": "k_yc_p<float,128>", "system_applications": 32, "launches": 2, "avg_launch_ms": 1.0,
         "bytes_per_system_application": 1e6}
    bench.attach_traffic(r, 16)
    assert r["traffic"] == round(t["full_dispatch_bytes"] / 16 * 32 / 2)
    assert r["valu_issue"]["instr_per_launch"] == round(2e8 / 16 * 32 / 2)
    # a summary of other sources reports nothing
    f.write_text(f.read_text().replace(bench.source_digest(), "0" * 64))
    assert bench.measured_traffic("k_yc_p<float,128>", 16) is None
    assert bench.measured_sq("k_yc_p<float,128>", 16) is None
