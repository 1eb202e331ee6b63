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
        assert bench.kernel_symbol(bf.BF_FP32_3M, bench.launched_schedule(bf.BF_FP32_3M, s), 7) == \
            "apply_fp32_3m16_ws"
    # store fields 6 to 9 run the FP32 forms on 16 x 16 tiles
    assert bench.kernel_symbol(bf.BF_FP32, 3, 7) == "apply_fp32_4m16_ws"
    assert bench.kernel_symbol(bf.BF_FP32, 3, 5) == "apply_fp32_ws"
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


def test_roof_follows_issued_work():
    """The roof is the larger of the issued matrix-core time and the HBM
    time: the four-product FP32 form at full width is matrix-core bound
    (issues 4 x 2 x 64 x 64 x 36 flops per product), the three-product form
    issues a quarter less and is HBM-bound, and the 16-bit forms are
    HBM-bound even with three split products."""
    from paper_1810_11451_amd import workloads as wl
    b = wl.single_w_batch(n=4)
    b.f[:] = 36
    assert bench.issued_flops(b, bf.BF_FP32) == 4 * 4 * 2 * 64 * 64 * 36
    assert bench.issued_flops(b, bf.BF_FP32_3M) == 4 * 3 * 2 * 64 * 64 * 36
    assert bench.issued_flops(b, bf.BF_FP16X2) == 4 * 3 * 2 * 128 * 64 * 80
    full = wl.full_width_batch(n=64)
    fl = {p: bench.roof_floors_us(full, p) for p in (bf.BF_FP32, bf.BF_FP32_3M, bf.BF_FP16X2)}
    assert fl[bf.BF_FP32]["compute_us"] > fl[bf.BF_FP32]["hbm_us"]
    assert fl[bf.BF_FP32_3M]["compute_us"] < fl[bf.BF_FP32_3M]["hbm_us"]
    assert fl[bf.BF_FP16X2]["compute_us"] < fl[bf.BF_FP16X2]["hbm_us"]


def test_buffer_sets_keep_s_out_of_the_memory_side_cache():
    """The timed workloads rotate enough disjoint buffer sets that their S
    is at least twice the 256 MB memory-side cache (at most 16 sets), so no
    launch reads S an earlier launch left there."""
    from paper_1810_11451_amd import workloads as wl

    def s_bytes(b):
        return int(b.f.astype("int64").sum()) * wl.B * 8

    for b in (wl.full_width_batch(), wl.uneven_batch(), wl.gain_batch()):
        n = bench.buffer_sets(b, 3)
        assert n >= 3 and n * s_bytes(b) >= 2 * bench.MALL_BYTES, (b.name, n)
        assert (n - 1) * s_bytes(b) < 2 * bench.MALL_BYTES or n == 3
    assert bench.buffer_sets(wl.uneven_batch(), 3) == 8
    assert bench.buffer_sets(wl.full_width_batch(), 3) == 3
    assert bench.buffer_sets(wl.single_w_batch(), 3) == 16     # capped: launch-bound anyway
    assert bench.buffer_sets(wl.uneven_batch(), 10) == 10      # never fewer than asked
