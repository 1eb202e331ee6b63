"""Environment settings of libbf, read when a plan is made (include/bf.h,
"Environment"): BF_FORCE_VARIANT overrides the variant of every launch,
BF_LOG reports plans and launch configurations on stderr, and
BF_AUTOTUNE_CACHE is the tuning database a plan loads and bf_autotune
writes.  Results are checked against the FP64 oracle under every setting.
"""
import numpy as np
import pytest

from gpu_util import FP32_TOL, announce, rel_errors, require_gpu
from paper_1810_11451_amd import bf
from paper_1810_11451_amd import workloads as wl
from paper_1810_11451_amd.device import DeviceBatch

pytestmark = pytest.mark.gpu


def _apply(plan, b, prec=bf.BF_FP32):
    db = DeviceBatch(b)
    db.apply(plan, prec)
    return db.result()


def test_force_variant_and_log(monkeypatch, capfd):
    require_gpu()
    monkeypatch.setenv("BF_LOG", "1")
    monkeypatch.setenv("BF_FORCE_VARIANT", "2:1:0:0")
    b = wl.uneven_batch(n=600)
    announce("BF_FORCE_VARIANT=2:1:0:0 BF_LOG=1")
    plan = bf.bf_plan_create(b.W)
    R = _apply(plan, b)
    plan.close()
    err = capfd.readouterr().err
    assert "[bf] plan: 256 W of 64 x 36" in err and "BF_FORCE_VARIANT set" in err
    assert "apply fp32 variant 2:1:0:0 -> schedule 2 grid" in err
    e, _ = rel_errors(b, R)
    assert np.max(e) <= FP32_TOL


def test_bad_force_variant_is_reported_and_ignored(monkeypatch, capfd):
    require_gpu()
    monkeypatch.setenv("BF_FORCE_VARIANT", "3:0:0:10")   # store 10 does not exist
    monkeypatch.delenv("BF_LOG", raising=False)
    b = wl.uneven_batch(n=300)
    plan = bf.bf_plan_create(b.W)
    R = _apply(plan, b)
    plan.close()
    assert 'BF_FORCE_VARIANT="3:0:0:10" ignored' in capfd.readouterr().err
    e, _ = rel_errors(b, R)
    assert np.max(e) <= FP32_TOL


def test_autotune_cache_is_written_and_loaded(monkeypatch, tmp_path):
    require_gpu()
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BF_AUTOTUNE_CACHE", str(path))
    monkeypatch.delenv("BF_FORCE_VARIANT", raising=False)
    b = wl.uneven_batch(n=1500)
    plan = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32_3M))
    db = DeviceBatch(b)
    announce("BF_AUTOTUNE_CACHE")
    best, us = bf.bf_autotune(plan, b.w_ids, b.f, db.s_ptrs[0], db.r_ptrs[0], prec=bf.BF_FP32_3M, reps=1)
    plan.close()
    assert path.exists() and us > 0
    bucket = bf.batch_bucket(b.f)
    plan2 = bf.bf_plan_create(b.W, bf.BF_PREC_BIT(bf.BF_FP32_3M))
    assert bf.bf_get_variant(plan2, bf.BF_FP32_3M, bucket) == best
    q_v, q_us = bf.bf_tune_query(plan2, bf.BF_FP32_3M, int(round(float(np.mean(b.f)))))
    assert q_v == best and abs(q_us - us) < 0.01
    R = _apply(plan2, b, bf.BF_FP32_3M)
    plan2.close()
    e, _ = rel_errors(b, R)
    assert np.max(e) <= FP32_TOL
