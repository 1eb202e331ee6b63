"""Host-side helpers of bench.py (CPU only): which kernel a variant runs,
and that recorded traffic is only used for that kernel and launch variant."""
import json

import bench
from paper_1810_11451_amd import bf


def test_launched_schedule_and_symbol():
    # the three-product form has one-per-workgroup and wave-specialised kernels only
    assert bench.kernel_symbol(bf.BF_FP32_3M, bench.launched_schedule(bf.BF_FP32_3M, 0)) == \
        "apply_fp32_3m_single"
    for s in (1, 2, 3):
        assert bench.kernel_symbol(bf.BF_FP32_3M, bench.launched_schedule(bf.BF_FP32_3M, s)) == \
            "apply_fp32_ws"
    # the 16-bit forms have no claim schedule
    for p in (bf.BF_FP16, bf.BF_BF16, bf.BF_FP16X2, bf.BF_BF16X2):
        assert bench.kernel_symbol(p, bench.launched_schedule(p, 1)) == "apply_lp_stream"
        assert bench.kernel_symbol(p, bench.launched_schedule(p, 3)) == "apply_lp_ws"
    assert bench.kernel_symbol(bf.BF_FP32, 1) == "apply_fp32_claim"


def test_traffic_entry_requires_matching_kernel(tmp_path, monkeypatch):
    entry = {"kernel_sha": bench.kernel_sha("configX-fp32"), "kernel": "apply_fp32_ws",
             "variant": "3:0:0:2", "traffic_bytes_per_launch": 123}
    root = tmp_path
    (root / "profiles").mkdir()
    (root / "profiles" / "traffic.json").write_text(json.dumps({"configX-fp32": entry}))
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.load_traffic("configX-fp32", "apply_fp32_ws") == 123
    assert bench.load_traffic("configX-fp32", "apply_fp32_single") is None
    assert bench.load_traffic("configY-fp32", "apply_fp32_ws") is None
    # the variant the counters were taken on must match the launched one
    assert bench.load_traffic("configX-fp32", "apply_fp32_ws", (3, 0, 0, 2)) == 123
    assert bench.load_traffic("configX-fp32", "apply_fp32_ws", (3, 0, 0, 1)) is None


def test_more_than_one_gpu_is_refused(capsys):
    """The library uses one GPU: --gpus N > 1 exits with status 2 and says why,
    before touching a device."""
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_workload_names():
    """Workloads are named by what they are; each batch generator exists."""
    assert set(bench.WORKLOADS) == {"single-w", "full-width", "uneven", "gain", "serving", "filter"}
    for name, gen in bench.WORKLOADS.items():
        assert (gen is None) == (name in ("serving", "filter"))
