"""The serving loop on the host executor: libbf's batcher, admission and
completion logic linked to a null device with a settable clock (no GPU).

These check the loop's own rules (include/bf.h, serving section): arrival
order, the HBM budget, one launch in flight per stream, the item bound per
launch, deadlines measured from arrival, early closing of launches against
the throughput estimate, failure reporting, drain on destroy, and the S and
R addresses the loop derives for each block of a request.
"""
import threading
import time

import numpy as np
import pytest

from paper_1810_11451_amd import bf
from paper_1810_11451_amd import hostexec as hx

M, B = bf.BF_M, bf.BF_B
BLOCK_R = M * B * 8


def req_bytes(f, n_s):
    return n_s * (f * B * 8 + BLOCK_R)


class Arena:
    """Host S and R memory for a list of (w_id, f, n_s) requests: every
    request gets its own S blocks (random values) and R blocks."""

    def __init__(self, specs, seed=0):
        rng = np.random.default_rng(seed)
        self.specs = specs
        s_len = sum(f * n_s * B for _, f, n_s in specs) + 2
        r_len = sum(n_s for _, _, n_s in specs)
        self.S = (rng.standard_normal(s_len) + 1j * rng.standard_normal(s_len)).astype(np.complex64)
        self.R = np.full((max(r_len, 1), M, B), np.nan + 1j * np.nan, np.complex64)
        self.reqs = np.zeros(len(specs), bf.REQUEST_DTYPE)
        so, ro = 0, 0
        self.s_at, self.r_at = [], []
        for i, (w, f, n_s) in enumerate(specs):
            self.reqs[i]["w_id"], self.reqs[i]["f"], self.reqs[i]["n_s"] = w, f, n_s
            self.reqs[i]["S"] = self.S.ctypes.data + so * 8 if f > 0 else 0
            self.reqs[i]["R"] = self.R.ctypes.data + ro * BLOCK_R
            self.reqs[i]["tag"] = i
            self.s_at.append(so)
            self.r_at.append(ro)
            so += f * n_s * B
            ro += n_s

    def check_marks(self, i):
        """The marks the null device writes for request i (see bfh_mark)."""
        w, f, n_s = self.specs[i]
        for k in range(n_s):
            blk = self.R[self.r_at[i] + k]
            assert blk[0, 0] == np.complex64(w + 1j * f)
            assert blk[M - 1, B - 1] == np.complex64(w + 1j * f)
            if f > 0:
                s0 = self.s_at[i] + k * f * B
                assert blk[0, 1] == self.S[s0]
                assert blk[0, 2] == self.S[s0 + f * B - 1]
            else:
                assert blk[0, 1] == 0 and blk[0, 2] == 0
            assert np.all(np.isnan(blk.reshape(-1)[3:-1].real)), "only the marks are written"


def wait_for(pred, timeout_s=10.0):
    """Waits until pred() holds (the loop's threads act asynchronously)."""
    t_end = time.monotonic() + timeout_s
    while not pred():
        assert time.monotonic() < t_end, "condition not reached"
        time.sleep(0.001)


def drain(srv, n, timeout_s=10.0):
    got = []
    t_end = time.monotonic() + timeout_s
    while sum(len(g) for g in got) < n:
        assert time.monotonic() < t_end, "completions did not arrive"
        got.append(srv.poll(1024, timeout_us=20000))
    return np.concatenate(got) if got else np.zeros(0, bf.COMPLETION_DTYPE)


def random_specs(rng, n, n_w=16, f_hi=36, ns_hi=8):
    return [(int(rng.integers(0, n_w)), int(rng.integers(0, f_hi + 1)), int(rng.integers(1, ns_hi + 1)))
            for _ in range(n)]


def test_every_request_completes_once_with_its_own_blocks():
    rng = np.random.default_rng(1)
    specs = random_specs(rng, 400)
    ar = Arena(specs, seed=1)
    dev = hx.Device(write_marks=True, launch_ns=20000, bytes_per_ns=2000.0)
    srv = hx.Server(dev, n_w=16, n_streams=3, max_batch_items=64)
    tickets = [srv.submit(ar.reqs[i]) for i in range(len(specs))]
    done = drain(srv, len(specs))
    st = srv.stats()
    srv.close()
    assert sorted(done["ticket"].tolist()) == sorted(tickets)
    assert np.all(done["status"] == bf.BF_OK)
    assert sorted(done["tag"].tolist()) == list(range(len(specs)))
    for i in range(len(specs)):
        ar.check_marks(i)
    L = dev.launches()
    assert np.all(L["n_items"] <= 64)
    assert int(L["n_reqs"].sum()) == len(specs)
    seen = np.concatenate([dev.launch_tickets(k) for k in range(len(L))])
    assert sorted(seen.tolist()) == sorted(tickets), "each request in exactly one launch"
    # requests enter launches in arrival (ticket) order
    assert np.all(np.diff(seen.astype(np.int64)) > 0)
    assert st["submitted"] == st["admitted"] == st["completed"] == len(specs)
    assert st["launches"] == len(L) and st["inflight_bytes"] == 0 and st["queued"] == 0
    assert dev.peak_unfinished() <= 6          # (two per stream under load)
    dev.close()


def test_budget_bounds_admission_and_waits_for_completions():
    f, n_s = 36, 2
    nb = req_bytes(f, n_s)
    ar = Arena([(0, f, n_s)] * 10)
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=1, hbm_budget_bytes=3 * nb, n_streams=2)
    for i in range(10):
        srv.submit(ar.reqs[i])
    wait_for(lambda: srv.stats()["admitted"] == 3 and len(dev.launches()) >= 1)
    time.sleep(0.02)                          # (and no more than 3)
    st = srv.stats()
    assert st["admitted"] == 3 and st["inflight_bytes"] == 3 * nb
    L = dev.launches()
    # the admitted three are launched as streams free up (two streams)
    assert 1 <= len(L) <= 2 and int(L["n_reqs"].sum()) <= 3
    assert srv.poll(16, 0).size == 0
    # completing frees budget; the loop admits and launches the next ones
    done = []
    while len(done) < 10:
        for s in range(2):
            dev.complete(s, 1)
        time.sleep(0.005)
        done.extend(srv.poll(16, 0).tolist())
        assert srv.stats()["inflight_bytes"] <= 3 * nb
    st = srv.stats()
    assert st["peak_inflight_bytes"] <= 3 * nb
    srv.close()
    dev.close()


def test_one_launch_in_flight_per_stream_under_light_load():
    """While the admitted work would not fill half a launch, a stream takes
    a new launch only when its previous one has finished."""
    ar = Arena([(0, 8, 1)] * 20)
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=1, n_streams=2, max_batch_items=64)
    for i in range(20):
        srv.submit(ar.reqs[i])
    wait_for(lambda: len(dev.launches()) == 2)
    time.sleep(0.02)                          # (and no third while both streams are busy)
    assert dev.unfinished(0) == 1 and dev.unfinished(1) == 1
    n = 0
    while n < 20:
        for s in range(2):
            dev.complete(s, 1)
        time.sleep(0.003)
        n += srv.poll(64, 0).size
        assert dev.unfinished(0) <= 1 and dev.unfinished(1) <= 1
    srv.close()
    assert int(dev.launches()["n_items"].sum()) == 20
    assert dev.peak_unfinished() == 2
    dev.close()


def test_two_launches_in_flight_per_stream_under_load():
    """With at least half a launch of work admitted, each stream also takes
    a second launch behind the running one, never a third."""
    ar = Arena([(0, 8, 1)] * 40)
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=1, n_streams=2, max_batch_items=4)
    for i in range(40):
        srv.submit(ar.reqs[i])
    wait_for(lambda: len(dev.launches()) == 4)
    time.sleep(0.02)                          # (and no fifth)
    assert dev.unfinished(0) == 2 and dev.unfinished(1) == 2
    L = dev.launches()
    assert len(L) == 4 and sorted(L["stream"].tolist()) == [0, 0, 1, 1]
    n = 0
    while n < 40:
        for s in range(2):
            dev.complete(s, 1)
        time.sleep(0.003)
        n += srv.poll(64, 0).size
        assert dev.unfinished(0) <= 2 and dev.unfinished(1) <= 2
    srv.close()
    L = dev.launches()
    # launches start as soon as a stream has room, so the first ones may be
    # smaller; none exceeds the item bound and together they cover all 40
    assert np.all(L["n_items"] <= 4) and int(L["n_items"].sum()) == 40
    assert np.sum(L["n_items"] == 4) >= len(L) - 5
    assert dev.peak_unfinished() == 4
    dev.close()


def test_submit_batch_checks_all_then_queues_what_fits():
    """bfh_submit_batch: a bad request anywhere queues nothing; with a
    small queue the call takes the prefix that fits (consecutive tickets),
    and the rest goes in later calls; every request completes once."""
    rng = np.random.default_rng(5)
    specs = random_specs(rng, 50)
    ar = Arena(specs, seed=5)
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=16, n_streams=2, queue_capacity=16)
    bad = ar.reqs[:10].copy()
    bad[7]["w_id"] = 99
    with pytest.raises(bf.BfError, match="request 7"):
        srv.submit_batch(bad)
    assert srv.stats()["submitted"] == 0
    n, first = srv.submit_batch(ar.reqs[:40])
    assert 1 <= n <= 16 and first == 1
    assert srv.stats()["refused"] == 1
    tickets = list(range(first, first + n))
    done = []
    i = n
    t_end = time.monotonic() + 10
    while len(done) < len(specs):
        assert time.monotonic() < t_end
        if i < len(specs):
            k, f0 = srv.submit_batch(ar.reqs[i:])
            if k:
                assert f0 == tickets[-1] + 1
                tickets.extend(range(f0, f0 + k))
                i += k
        for s in range(2):
            dev.complete(s, 1)
        done.extend(srv.poll(64, 1000).tolist())
    srv.close()
    dev.close()
    d = np.array(done, bf.COMPLETION_DTYPE)
    assert sorted(d["ticket"].tolist()) == tickets == list(range(1, len(specs) + 1))
    assert sorted(d["tag"].tolist()) == list(range(len(specs)))


def test_deadline_is_measured_from_arrival():
    ar = Arena([(0, 4, 1)] * 3)
    dev = hx.Device(manual_clock=True, manual_complete=True)
    srv = hx.Server(dev, n_w=1, n_streams=1, deadline_us=500)
    t0 = dev.clock_now()
    r = ar.reqs.copy()
    r["t_arrival_ns"] = [t0, t0, t0 - 400_000]     # the third arrived 400 us before submit
    srv.submit(r[0])
    wait_for(lambda: len(dev.launches()) == 1)
    dev.clock_set(t0 + 499_000)
    dev.complete(0, 1)
    a = drain(srv, 1)
    srv.submit(r[1])
    srv.submit(r[2])
    wait_for(lambda: srv.stats()["admitted"] == 3 and len(dev.launches()) >= 2)
    dev.clock_set(t0 + 600_000)
    got = []
    t_end = time.monotonic() + 10
    while len(got) < 2:                       # (one launch or two, as they were taken)
        assert time.monotonic() < t_end
        dev.complete(0, 1)
        got.extend(srv.poll(4, 2000).tolist())
    b = np.array(got, bf.COMPLETION_DTYPE)
    st = srv.stats()
    srv.close()
    dev.close()
    assert a["deadline_missed"][0] == 0 and a["t_done_ns"][0] == t0 + 499_000
    by_tag = {int(c["tag"]): c for c in b}
    assert by_tag[1]["deadline_missed"] == 1 and by_tag[2]["deadline_missed"] == 1
    assert by_tag[2]["t_arrival_ns"] == t0 - 400_000
    assert st["deadline_misses"] == 2


def test_launch_closed_early_to_keep_the_oldest_deadline():
    # One large launch teaches the loop its throughput (launches of 8 MiB or
    # more are measured), then a queue builds up behind a busy stream: the
    # next launch takes only what is predicted to finish by the oldest
    # member's deadline.
    big = [(0, 36, 256)]                     # 8.3 MB
    small = [(0, 36, 16)] * 12               # 0.52 MB each
    ar = Arena(big + small)
    dev = hx.Device(manual_clock=True, manual_complete=True)
    srv = hx.Server(dev, n_w=1, n_streams=1, deadline_us=500)
    t0 = dev.clock_now()
    srv.submit(ar.reqs[0])
    wait_for(lambda: len(dev.launches()) == 1)
    nb = req_bytes(36, 256)
    dev.clock_set(t0 + nb // 4)              # finishes at 4 bytes per ns
    dev.complete(0, 1)
    drain(srv, 1)
    # a launch in flight keeps the stream busy while the queue builds
    srv.submit(ar.reqs[1])
    wait_for(lambda: len(dev.launches()) == 2)
    t1 = dev.clock_now()
    rest = ar.reqs[2:].copy()
    rest["t_arrival_ns"] = t1                # 500 us left for each
    for q in rest:
        srv.submit(q)
    wait_for(lambda: srv.stats()["admitted"] == 13)
    dev.complete(0, 1)                       # frees the stream; nothing else moves the clock
    wait_for(lambda: len(dev.launches()) == 3)
    L = dev.launches()
    srv_stats = srv.stats()
    # rate 4 B/ns x 500 us = 2 MB: at most 3 of the 0.52 MB requests (the first always goes)
    third = L[2]
    assert third["n_reqs"] == int(min(11, max(1, (4 * 500_000) // req_bytes(36, 16))))
    t_end = time.monotonic() + 10
    while srv_stats["completed"] < 13:
        assert time.monotonic() < t_end
        dev.complete(0, 1)
        time.sleep(0.002)
        srv_stats = srv.stats()
    srv.close()
    dev.close()


def test_failed_launch_reports_its_requests_and_the_server():
    ar = Arena([(0, 8, 1)] * 6)
    dev = hx.Device(manual_complete=True)
    dev.fail_launch(1, bf.BF_ERR_DEVICE)
    srv = hx.Server(dev, n_w=1, n_streams=1, max_batch_items=2)
    for i in range(6):
        srv.submit(ar.reqs[i])
    got = []
    t_end = time.monotonic() + 5
    while len(got) < 6:
        assert time.monotonic() < t_end
        dev.complete(0, 1)
        got.extend(srv.poll(16, 2000).tolist())
    status = {int(c[0]): int(c[2]) for c in got}              # ticket -> status
    failed = set(dev.launch_tickets(1).tolist())               # the launch made to fail
    assert len(failed) >= 1
    assert all(status[t] == (bf.BF_ERR_DEVICE if t in failed else bf.BF_OK) for t in status)
    assert dev.launches()["status"][1] == bf.BF_ERR_DEVICE
    with pytest.raises(bf.BfError) as e:
        srv.close()
    assert e.value.status == bf.BF_ERR_DEVICE
    dev.close()


def test_device_error_at_completion_is_reported():
    ar = Arena([(0, 8, 1)] * 2)
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=1, n_streams=1, max_batch_items=1)
    srv.submit(ar.reqs[0])
    srv.submit(ar.reqs[1])
    wait_for(lambda: len(dev.launches()) >= 1)     # (the second may queue behind it)
    dev.complete(0, 1, bf.BF_ERR_DEVICE)
    a = drain(srv, 1)
    wait_for(lambda: len(dev.launches()) == 2)
    dev.complete(0, 1)
    b = drain(srv, 1)
    assert a["status"][0] == bf.BF_ERR_DEVICE and b["status"][0] == bf.BF_OK
    with pytest.raises(bf.BfError):
        srv.close()
    dev.close()


def test_destroy_drains_everything_submitted():
    rng = np.random.default_rng(3)
    specs = random_specs(rng, 300, ns_hi=4)
    ar = Arena(specs)
    dev = hx.Device(launch_ns=50_000, bytes_per_ns=500.0, write_marks=True)
    srv = hx.Server(dev, n_w=16, n_streams=2, max_batch_items=32)
    for i in range(len(specs)):
        srv.submit(ar.reqs[i])
    srv.close()                               # returns only once all have run
    L = dev.launches()
    assert int(L["n_reqs"].sum()) == len(specs) and np.all(L["status"] == 0)
    for i in range(len(specs)):
        ar.check_marks(i)
    assert dev.unfinished() == 0
    dev.close()


def test_full_queue_refuses_and_bad_requests_are_rejected():
    ar = Arena([(0, 8, 1)] * 8 + [(0, 36, 1)])
    dev = hx.Device(manual_complete=True)
    srv = hx.Server(dev, n_w=2, f_max=20, hbm_budget_bytes=req_bytes(8, 1), n_streams=1,
                    queue_capacity=4)
    # the first is admitted and launched; the rest wait for budget in the
    # loop's own queue, so the submission ring fills only once that has
    # taken what it can: submit until refused
    busy = 0
    for i in range(8):
        try:
            srv.submit(ar.reqs[i])
        except bf.BfError as e:
            assert e.status == bf.BF_ERR_BUSY
            busy += 1
    bad = []
    r = ar.reqs[0].copy()
    r["w_id"] = 2
    bad.append(r)
    r = ar.reqs[8].copy()                     # f = 36 > f_max = 20
    bad.append(r)
    r = ar.reqs[0].copy()
    r["n_s"] = 0
    bad.append(r)
    r = ar.reqs[0].copy()
    r["R"] += 8                               # 8-byte aligned only
    bad.append(r)
    r = ar.reqs[0].copy()
    r["n_s"] = 2                              # larger than the whole budget
    bad.append(r)
    for q in bad:
        with pytest.raises(bf.BfError) as e:
            srv.submit(q)
        assert e.value.status == bf.BF_ERR_INVALID
    n_ok = srv.stats()["submitted"]
    assert srv.stats()["refused"] == busy and n_ok + busy == 8
    got = 0
    t_end = time.monotonic() + 5
    while got < n_ok:
        assert time.monotonic() < t_end
        dev.complete(0, 1)
        got += srv.poll(16, 2000).size
    srv.close()
    dev.close()


def test_bad_config_is_rejected():
    dev = hx.Device()
    for kw in ({"hbm_budget_bytes": 0}, {"n_streams": 0}, {"n_streams": 9}, {"max_batch_items": 0},
               {"queue_capacity": 3}):
        with pytest.raises(bf.BfError) as e:
            hx.Server(dev, n_w=1, **kw)
        assert e.value.status == bf.BF_ERR_INVALID
    dev.close()


def test_poisson_replay_in_real_time_finishes():
    """Two streams, mixed f and S counts, Poisson arrivals paced in real
    time against a device model at a fixed rate: every request finishes and
    the latency (from the submit; this Python pacer cannot hold a schedule
    to the microsecond) stays near the model's service time."""
    rng = np.random.default_rng(5)
    n = 2000
    specs = [(int(rng.integers(0, 64)), int(rng.integers(1, 37)), int(rng.integers(1, 9)))
             for _ in range(n)]
    ar = Arena(specs)
    dev = hx.Device(launch_ns=10_000, bytes_per_ns=400.0)
    srv = hx.Server(dev, n_w=64, n_streams=2, deadline_us=500)
    gaps = rng.exponential(1e9 / 5000.0, n)             # 5k req/s offered
    t_sched = np.cumsum(gaps).astype(np.int64)
    got = []
    count = [0]

    def poller():
        t_end = time.monotonic() + 30
        while count[0] < n and time.monotonic() < t_end:
            c = srv.poll(1024, 20000)
            if c.size:
                got.append(c)
                count[0] += c.size

    th = threading.Thread(target=poller)
    th.start()
    t0 = time.monotonic_ns()
    for i in range(n):
        while time.monotonic_ns() - t0 < t_sched[i]:
            time.sleep(0)
        srv.submit(ar.reqs[i])
    th.join(timeout=40)
    assert not th.is_alive() and count[0] == n, "replay stalled"
    done = np.concatenate(got)
    srv.close()
    dev.close()
    assert np.all(done["status"] == 0)
    lat_us = (done["t_done_ns"] - done["t_arrival_ns"]) / 1e3
    # service time of the largest request: 10 us + 8 x 48 KB at 400 B/ns = 1 ms
    assert np.all(lat_us > 0) and np.percentile(lat_us, 50) < 1000
