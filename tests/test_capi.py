"""The C-ABI library on the CPU: it loads, exports every entry point that
include/tdct.h declares, reports argument errors before touching a device,
and its server logic (admission under a budget, FIFO order, batching,
failure handling, drain) runs against the fake device."""
import ctypes
import os
import re
import time

import numpy as np
import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "tdct.h")


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tdct_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol(tdct):
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(tdct.lib(), n)]
    assert not missing, missing


def test_binding_names_match_the_abi(tdct):
    skip = {"tdct_plan_free", "tdct_server_destroy"}
    for n in _declared():
        assert hasattr(tdct, n) or n in skip, n


def test_strerror_covers_every_status(tdct):
    for st in range(0, -8, -1):
        assert tdct.tdct_strerror(st) != "unknown status"
    assert tdct.tdct_strerror(-99) == "unknown status"


def test_argument_errors_need_no_device(tdct):
    L = tdct.lib()
    q = tdct.qtable(np.ones(64))
    fake = 0x10000  # never dereferenced: validation fails first
    r = ctypes.byref
    assert L.tdct_quantise(fake, 8, 7, 8, r(q), 64, fake, None) == tdct.TDCT_EDIM
    assert L.tdct_quantise(fake, 8, 8, 65544, r(q), 64, fake, None) == tdct.TDCT_EDIM
    assert L.tdct_forward(None, 8, 8, 8, fake, None) == tdct.TDCT_EINVAL
    assert L.tdct_inverse(fake + 4, r(q), 8, 8, fake, 8, None) == tdct.TDCT_EINVAL
    assert L.tdct_roundtrip(fake, 8, 8, 8, r(q), 64, fake + 8, fake, 8, None) == tdct.TDCT_EINVAL
    bad = tdct.qtable(np.ones(64))
    bad.q[63] = 4096
    assert L.tdct_quantise_i8_zigzag(fake, 8, 8, 8, r(bad), fake, None) == tdct.TDCT_EQTAB
    assert L.tdct_sse(fake, 8, fake, 8, 8, 8, None, None) == tdct.TDCT_EINVAL
    d = tdct.image_desc(tdct.OP_ENCODE, 16, 16, qtab=3, keep=64, src=fake, src_stride=16, coef=fake)
    h = ctypes.c_void_p()
    qa = (tdct.tdct_qtable * 1)(q)
    assert L.tdct_batch_plan((tdct.tdct_image_desc * 1)(d), 1, qa, 1, None, r(h)) == tdct.TDCT_EINVAL
    d.qtab, d.keep = 0, 0
    assert L.tdct_batch_plan((tdct.tdct_image_desc * 1)(d), 1, qa, 1, None, r(h)) == tdct.TDCT_EINVAL
    d.keep, d.op = 64, 9
    assert L.tdct_batch_plan((tdct.tdct_image_desc * 1)(d), 1, qa, 1, None, r(h)) == tdct.TDCT_EINVAL
    d.op = tdct.OP_ENCODE
    for bad_tune in ((3, 1, 1, 0, 0), (16, 1, 1, 0, 0), (4, 5000, 1, 0, 0), (4, 1, 3, 0, 0),
                     (4, 1, 1, 2, 0), (4, 1, 1, 0, 2), (4, 1, 1, 0, -1)):
        t = tdct.tdct_tune(*bad_tune)
        assert L.tdct_batch_plan((tdct.tdct_image_desc * 1)(d), 1, qa, 1, r(t), r(h)) == tdct.TDCT_EINVAL


def test_plans_refuse_outputs_over_inputs(tdct):
    """A plan runs many times (graph replays, autotuning), so an image may not
    write bytes any image of the plan reads: an in-place round trip, a decode
    of coefficients the same plan encodes, or an output plane reaching into
    another image's rows are refused before any device is touched."""
    L = tdct.lib()
    qa = (tdct.tdct_qtable * 1)(tdct.qtable(np.ones(64)))
    h = ctypes.c_void_p()

    def plan(*descs):
        arr = (tdct.tdct_image_desc * len(descs))(*descs)
        return L.tdct_batch_plan(arr, len(descs), qa, 1, None, ctypes.byref(h))

    a, b, c = 1 << 32, 2 << 32, 3 << 32
    rt = tdct.image_desc(tdct.OP_ROUNDTRIP, 64, 64, src=a, src_stride=64, dst=a, dst_stride=64)
    assert plan(rt) == tdct.TDCT_EINVAL
    enc = tdct.image_desc(tdct.OP_ENCODE, 64, 64, src=a, src_stride=64, coef=b)
    dec = tdct.image_desc(tdct.OP_DECODE, 64, 64, coef=b + 128 * 63, dst=c, dst_stride=64)
    assert plan(enc, dec) == tdct.TDCT_EINVAL
    # the last row of a strided plane ends at (h - 1) * stride + w
    enc2 = tdct.image_desc(tdct.OP_ENCODE, 64, 64, src=c + 63 * 100 + 63, src_stride=100, coef=b)
    dec2 = tdct.image_desc(tdct.OP_DECODE, 64, 64, coef=a, dst=c, dst_stride=100)
    assert plan(enc2, dec2) == tdct.TDCT_EINVAL
    # adjacent spans do not meet: validation passes, and the missing device
    # (or a real one) decides the rest
    dec3 = tdct.image_desc(tdct.OP_DECODE, 64, 64, coef=b + 128 * 64, dst=c, dst_stride=64)
    assert plan(enc, dec3) != tdct.TDCT_EINVAL
    if h.value:
        L.tdct_plan_free(h)


def test_tune_cache_file_format(tdct, tmp_path):
    """The autotune cache opens a missing file as empty, reads the file
    format it writes, and refuses anything else (cache off). Lookups and
    stores need a device (GPU tests)."""
    path = str(tmp_path / "tune.json")
    try:
        tdct.tdct_tune_cache_open(path)
        info = tdct.tdct_tune_cache_info()
        assert info["on"] == 1 and info["entries"] == 0
        good = ('{"format": "tdct-autotune-1", "entries": {\n'
                '  "gfx950/src=0123456789abcdef/ops=1/tiles=17/aligned=1": [4, 1, 2, 1, 0],\n'
                '  "gfx950/src=0123456789abcdef/ops=2/tiles=18/aligned=1": [2, 4096, 1, 0, 1]\n}}\n')
        open(path, "w").write(good)
        tdct.tdct_tune_cache_open(path)
        assert tdct.tdct_tune_cache_info()["entries"] == 2
        open(path, "w").write('{"format": "tdct-autotune-1", "entries": {}}')
        tdct.tdct_tune_cache_open(path)
        assert tdct.tdct_tune_cache_info() ["entries"] == 0
        bad = [good.replace("[4, 1, 2", "[3, 1, 2"),           # waves per group not 1/2/4/8
               good.replace("[2, 4096, 1, 0, 1]", "[2, 4096, 1, 0]"),  # a field missing
               good.replace("tdct-autotune-1", "tdct-autotune-0"),
               good.replace('"entries"', '"entry"'),
               good[:-3],                                          # truncated
               good + "x",                                         # trailing bytes
               "[]"]
        for text in bad:
            open(path, "w").write(text)
            with pytest.raises(tdct.TdctError) as e:
                tdct.tdct_tune_cache_open(path)
            assert e.value.status == tdct.TDCT_EINVAL
            assert tdct.tdct_tune_cache_info()["on"] == 0
        tdct.tdct_tune_cache_open(path + ".missing")
        assert tdct.tdct_tune_cache_info()["on"] == 1
    finally:
        tdct.tdct_tune_cache_open(None)
    assert tdct.tdct_tune_cache_info()["on"] == 0


# ---- server logic on the fake device ----------------------------------------

def test_server_tune_is_validated(tdct):
    """The server's launch shape goes through the same checks as a plan's:
    out-of-range fields are rejected at create, zero fields take defaults."""
    for bad in (dict(waves_per_group=3), dict(tile_waves=8), dict(xcd_remap=-1),
                dict(pixel_cache=2)):
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_create(tdct.server_cfg(1 << 20, fake_device_us=100, tune=bad))
        assert e.value.status == tdct.TDCT_EINVAL
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 20, fake_device_us=100,
                                                tune=dict(xcd_remap=1, pixel_cache=1)))
    try:
        t = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 32))
        tdct.tdct_server_drain(s)
        assert tdct.tdct_server_poll(s, t).status == tdct.TDCT_OK
    finally:
        tdct.tdct_server_destroy(s)


def _req(tdct, op, w, h, keep=64):
    return tdct.request(op, w, h, 0x1000, np.ones(64), keep=keep)


def test_fake_server_completes_everything_and_counts(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 24, streams=2, max_batch=4, fake_device_us=200))
    try:
        tickets = [tdct.tdct_server_submit(s, _req(tdct, k % 2, 64, 32)) for k in range(20)]
        tdct.tdct_server_drain(s)
        for t in tickets:
            r = tdct.tdct_server_poll(s, t)
            assert r.status == tdct.TDCT_OK and r.output and r.done_us >= r.submit_us
            assert 1 <= r.batch_size <= 4
        st = tdct.tdct_server_stats(s)
        assert st["completed"] == 20 and st["failed"] == 0 and st["batches"] >= 5
        assert st["pixels_done"] == 20 * 64 * 32
        assert st["p50_us"] > 0 and st["p99_us"] >= st["p50_us"]
        for t in tickets:
            tdct.tdct_server_release(s, t)
        assert tdct.tdct_server_stats(s)["arena_bytes_in_use"] == 0
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_poll(s, tickets[0])
        assert e.value.status == tdct.TDCT_ENOTFOUND
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_launches_lone_requests_from_submit(tdct):
    """Requests spaced wider than the scheduler's polling window find it
    asleep; each is admitted and launched by the submitting thread and still
    completed by the scheduler, alone in its batch. Bursts in between go
    through the scheduler and batch as before."""
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 24, streams=2, max_batch=8, fake_device_us=300))
    try:
        lone = []
        for k in range(6):
            time.sleep(0.006)  # past the 2 ms polling window: the scheduler sleeps
            lone.append(tdct.tdct_server_submit(s, _req(tdct, k % 2, 64, 32)))
            assert tdct.tdct_server_wait(s, lone[-1]).status == tdct.TDCT_OK
        time.sleep(0.006)
        burst = [tdct.tdct_server_submit(s, _req(tdct, k % 2, 64, 32)) for k in range(24)]
        tdct.tdct_server_drain(s)
        for t in lone:
            r = tdct.tdct_server_poll(s, t)
            assert r.status == tdct.TDCT_OK and r.batch_size == 1 and r.done_us >= r.submit_us
        sizes = [tdct.tdct_server_poll(s, t).batch_size for t in burst]
        assert all(tdct.tdct_server_poll(s, t).status == tdct.TDCT_OK for t in burst)
        assert max(sizes) > 1  # the burst was batched
        st = tdct.tdct_server_stats(s)
        assert st["completed"] == 30 and st["failed"] == 0
        assert tdct.tdct_server_last_error(s) == ""
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_idle_poll_window(tdct):
    """idle_poll_us sets how long the scheduler polls after the last activity
    (0: 2 ms); out-of-range values are refused at create. With a window longer
    than the gaps between requests, spaced requests complete as before."""
    for bad in (-1, 10000001):
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_create(tdct.server_cfg(1 << 24, fake_device_us=100, idle_poll_us=bad))
        assert e.value.status == tdct.TDCT_EINVAL
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 24, streams=2, fake_device_us=200, idle_poll_us=50000))
    try:
        for k in range(5):
            time.sleep(0.006)
            t = tdct.tdct_server_submit(s, _req(tdct, k % 2, 64, 32))
            r = tdct.tdct_server_wait(s, t)
            assert r.status == tdct.TDCT_OK and r.batch_size == 1
        assert tdct.tdct_server_stats(s)["completed"] == 5
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_admission_never_exceeds_budget(tdct):
    budget = 3 * 64 * 64 * 2  # room for three encode outputs of 64 x 64
    s = tdct.tdct_server_create(tdct.server_cfg(budget, streams=4, max_batch=8, fake_device_us=300))
    try:
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 128, 128))
        assert e.value.status == tdct.TDCT_ENOMEM
        tickets = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64)) for _ in range(9)]
        done = []
        while len(done) < 9:
            for t in tickets:
                if t in done:
                    continue
                r = tdct.tdct_server_poll(s, t)
                if r.status == tdct.TDCT_OK:
                    done.append(t)
                    tdct.tdct_server_release(s, t)
            assert tdct.tdct_server_stats(s)["arena_high_water"] <= budget
            time.sleep(0.0005)
        # FIFO: the first three requests fit and run (in parallel, on three
        # stream slots, so their order among themselves is open); every later
        # one waits for a release
        assert sorted(done[:3]) == tickets[:3] and max(done[:3]) < min(done[3:])
        st = tdct.tdct_server_stats(s)
        assert st["arena_high_water"] <= budget and st["rejected"] == 1
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_failed_batches_do_not_stop_service(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 22, streams=1, max_batch=1, fake_device_us=100,
                                                fake_fail_every=3))
    try:
        tickets = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_DECODE, 32, 32)) for _ in range(9)]
        tdct.tdct_server_drain(s)
        status = [tdct.tdct_server_poll(s, t).status for t in tickets]
        assert status.count(tdct.TDCT_EDEVICE) == 3 and status.count(tdct.TDCT_OK) == 6
        st = tdct.tdct_server_stats(s)
        assert st["failed"] == 3 and st["completed"] == 6
        # failed requests gave their memory back
        for t, stt in zip(tickets, status):
            tdct.tdct_server_release(s, t)
        assert tdct.tdct_server_stats(s)["arena_bytes_in_use"] == 0
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_launch_failure_waits_for_queued_work(tdct):
    """A batch whose launch fails after part of its work was queued on the
    slot's stream gives its arena bytes and its slot back only once that work
    has drained (the fake device checks it), and the server goes on."""
    us = 3000
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 22, streams=1, max_batch=1, fake_device_us=us,
                                                fake_fail_every=-2))
    try:
        tickets = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_DECODE, 32, 32)) for _ in range(6)]
        tdct.tdct_server_drain(s)
        res = [tdct.tdct_server_poll(s, t) for t in tickets]
        status = [r.status for r in res]
        assert status.count(tdct.TDCT_EDEVICE) == 3 and status.count(tdct.TDCT_OK) == 3
        for r in res:  # failed or not, each request waited for its queued work
            assert r.done_us - r.submit_us >= us
        assert "released while" not in tdct.tdct_server_last_error(s)
        assert "after its work was queued" in tdct.tdct_server_last_error(s)
        for t in tickets:
            tdct.tdct_server_release(s, t)
        assert tdct.tdct_server_stats(s)["arena_bytes_in_use"] == 0
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_spreads_requests_over_free_slots(tdct):
    """Without a batching window a free slot takes ceil(admitted / slots)
    requests: requests that free slots can take one by one launch alone, and
    a backlog is shared out in batches of about equal size."""
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 24, streams=4, max_batch=16, fake_device_us=30000))
    try:
        first = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 32, 32)) for _ in range(4)]
        time.sleep(0.005)  # all four slots busy for 30 ms
        backlog = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 32, 32)) for _ in range(16)]
        tdct.tdct_server_drain(s)
        assert [tdct.tdct_server_poll(s, t).batch_size for t in first] == [1, 1, 1, 1]
        sizes = [tdct.tdct_server_poll(s, t).batch_size for t in backlog]
        assert max(sizes) == 4 and min(sizes) >= 1
        assert tdct.tdct_server_stats(s)["completed"] == 20
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_batches_requests_that_arrive_together(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 26, streams=1, max_batch=16, max_wait_us=20000,
                                                fake_device_us=100))
    try:
        tickets = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 32, 32)) for _ in range(16)]
        tdct.tdct_server_drain(s)
        sizes = {tdct.tdct_server_poll(s, t).batch_size for t in tickets}
        assert sizes == {16}
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_replay_and_shutdown_with_work_in_flight(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 24, streams=2, max_batch=8, fake_device_us=500))
    try:
        reqs = [_req(tdct, k % 2, 32, 64) for k in range(50)]
        arr = [k * 200.0 for k in range(50)]
        tk, lat, st = tdct.tdct_server_replay(s, reqs, arr)
        assert all(x == tdct.TDCT_OK for x in st) and min(lat) >= 500
        assert tdct.tdct_server_stats(s)["arena_bytes_in_use"] == 0
        for _ in range(10):
            tdct.tdct_server_submit(s, _req(tdct, 0, 64, 64))
    finally:
        tdct.tdct_server_destroy(s)  # drains the ten in flight, then stops


def test_failed_server_create_frees_what_it_built(tdct):
    """A fake-device server whose arena cannot be allocated (4 EiB) fails
    with TDCT_ENOMEM, in stream and in resident mode; its partly built state
    goes through the destroy path, and a server created afterwards works."""
    for resident in (0, 1):
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_create(tdct.server_cfg(1 << 62, fake_device_us=10, resident=resident))
        assert e.value.status == tdct.TDCT_ENOMEM
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 20, fake_device_us=10))
    try:
        t = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64))
        assert tdct.tdct_server_wait(s, t).status == tdct.TDCT_OK
    finally:
        tdct.tdct_server_destroy(s)


def test_server_rejects_bad_requests(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 20, fake_device_us=10))
    try:
        for r in (tdct.request(5, 8, 8, 0x1000, np.ones(64)), tdct.request(0, 12, 8, 0x1000, np.ones(64)),
                  tdct.request(0, 8, 8, None, np.ones(64)), tdct.request(1, 8, 8, 0x1008, np.ones(64)),
                  tdct.request(0, 8, 8, 0x1000, np.zeros(64))):
            with pytest.raises(tdct.TdctError):
                tdct.tdct_server_submit(s, r)
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_server_shutdown_with_unreleased_outputs_does_not_hang(tdct):
    """The second request can never be admitted (the first output is held by
    the client); destroying the server fails it instead of waiting forever."""
    import threading
    s = tdct.tdct_server_create(tdct.server_cfg(64 * 64 * 2, streams=1, max_batch=1, fake_device_us=50))
    t1 = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64))
    assert tdct.tdct_server_wait(s, t1).status == tdct.TDCT_OK
    t2 = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64))
    time.sleep(0.01)
    assert tdct.tdct_server_poll(s, t2).status == tdct.TDCT_EBUSY  # still waiting for memory
    th = threading.Thread(target=tdct.tdct_server_destroy, args=(s,))
    th.start()
    th.join(timeout=10)
    assert not th.is_alive()


def test_fake_server_pixel_cap_limits_batches(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 26, streams=1, max_batch=16, max_wait_us=20000,
                                                fake_device_us=100, max_batch_px=2 * 64 * 64))
    try:
        tickets = [tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64)) for _ in range(6)]
        big = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 256, 256))
        tdct.tdct_server_drain(s)
        assert {tdct.tdct_server_poll(s, t).batch_size for t in tickets} == {2}
        assert tdct.tdct_server_poll(s, big).batch_size == 1  # larger than the cap: alone
    finally:
        tdct.tdct_server_destroy(s)


def test_host_io_request_needs_a_host_output(tdct):
    s = tdct.tdct_server_create(tdct.server_cfg(1 << 20, fake_device_us=10))
    try:
        r = tdct.request(tdct.OP_DECODE, 8, 8, 0x1008, np.ones(64))
        r.host_io = 1  # no host_output
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_submit(s, r)
        assert e.value.status == tdct.TDCT_EINVAL
        ok = tdct.request(tdct.OP_DECODE, 8, 8, 0x1008, np.ones(64), host_output=0x2000)
        t = tdct.tdct_server_submit(s, ok)  # unaligned host input is fine: it is staged
        assert tdct.tdct_server_wait(s, t).output == 0x2000
    finally:
        tdct.tdct_server_destroy(s)


# ---- resident mode on the fake device ----------------------------------------
# A host thread plays the resident kernel's part of the queue protocol. It
# checks, before raising each done flag, that the request's queue slot and
# tile-ring entries were not reused early, and reports a violation through
# tdct_server_last_error.

def _resident(tdct, budget=1 << 26, **kw):
    kw.setdefault("fake_device_us", 100)
    return tdct.tdct_server_create(tdct.server_cfg(budget, resident=1, **kw))


def test_fake_resident_wraps_both_rings_without_reuse(tdct):
    # 4 queue slots and 16 tile slots; requests of 1 to 16 tiles (a tile is 128
    # blocks encoding, 64 decoding: 256 x 256 is 8 tiles encoded, 16 decoded)
    s = _resident(tdct, resident_jobs=4, resident_tiles=16, fake_device_us=60)
    try:
        sizes = [(64, 32), (256, 256), (128, 64), (256, 128), (32, 32), (256, 256), (64, 64)]
        tickets = []
        for k in range(60):
            w, h = sizes[k % len(sizes)]
            tickets.append(tdct.tdct_server_submit(s, _req(tdct, k % 2, w, h)))
        deadline = time.time() + 10  # a protocol fault shows as a request that never ends
        while tdct.tdct_server_stats(s)["completed"] < 60 and time.time() < deadline:
            time.sleep(0.002)
        assert tdct.tdct_server_last_error(s) == ""
        for t in tickets:
            r = tdct.tdct_server_poll(s, t)
            assert r.status == tdct.TDCT_OK and 1 <= r.batch_size <= 4
        st = tdct.tdct_server_stats(s)
        assert st["completed"] == 60 and st["failed"] == 0 and st["batches"] >= 1
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_resident_relaunches_after_idle_exit(tdct):
    s = _resident(tdct, resident_idle_us=1000, fake_device_us=50)
    try:
        t1 = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 64, 64))
        assert tdct.tdct_server_wait(s, t1).status == tdct.TDCT_OK
        time.sleep(0.02)  # well past the idle limit: the stand-in kernel has exited
        t2 = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_DECODE, 64, 64))
        assert tdct.tdct_server_wait(s, t2).status == tdct.TDCT_OK
        assert tdct.tdct_server_stats(s)["batches"] == 2  # two launches
        assert tdct.tdct_server_last_error(s) == ""
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_resident_refuses_what_it_cannot_serve(tdct):
    s = _resident(tdct, resident_tiles=8)
    try:
        t = tdct.tdct_server_submit(s, _req(tdct, tdct.OP_ENCODE, 256, 256))  # 8 tiles: fits
        assert tdct.tdct_server_wait(s, t).status == tdct.TDCT_OK
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_submit(s, _req(tdct, tdct.OP_DECODE, 256, 256))  # 16 tiles
        assert e.value.status == tdct.TDCT_ENOMEM
        assert tdct.tdct_server_stats(s)["rejected"] == 1
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_submit(s, tdct.request(tdct.OP_DECODE, 8, 8, 0x1008, np.ones(64),
                                                    host_output=0x2000))
        assert e.value.status == tdct.TDCT_EINVAL
    finally:
        tdct.tdct_server_destroy(s)


def test_fake_resident_replay_and_shutdown_with_work_in_flight(tdct):
    s = _resident(tdct, resident_jobs=8, fake_device_us=300)
    try:
        reqs = [_req(tdct, k % 2, 32, 64) for k in range(40)]
        tk, lat, st = tdct.tdct_server_replay(s, reqs, [k * 100.0 for k in range(40)])
        assert all(x == tdct.TDCT_OK for x in st) and min(lat) >= 300
        assert tdct.tdct_server_stats(s)["arena_bytes_in_use"] == 0
        for _ in range(10):
            tdct.tdct_server_submit(s, _req(tdct, 0, 64, 64))
    finally:
        tdct.tdct_server_destroy(s)  # the ten in flight finish first


# ---- diagnostics -------------------------------------------------------------

_LOG_SCRIPT = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import paper_1702_00817_amd as tdct
s = tdct.tdct_server_create(tdct.server_cfg(1 << 22, streams=1, max_batch=1, fake_device_us=200,
                                            fake_fail_every=3))
for k in range(6):
    tdct.tdct_server_submit(s, tdct.request(k % 2, 64, 32, 0x1000, np.ones(64)))
tdct.tdct_server_drain(s)
tdct.tdct_server_destroy(s)
print("level", tdct.tdct_log_level())
"""


@pytest.mark.parametrize("level", ["", "1", "2", "3"])
def test_log_levels_on_stderr(level):
    """TDCT_LOG sets the stderr diagnostics: nothing by default, errors at 1,
    server lifecycle at 2, every batch at 3 (fake device, injected failures)."""
    import subprocess
    import sys
    env = dict(os.environ)
    env.pop("TDCT_LOG", None)
    if level:
        env["TDCT_LOG"] = level
    r = subprocess.run([sys.executable, "-c", _LOG_SCRIPT, ROOT], env=env, stdin=subprocess.DEVNULL,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().endswith("level %d" % (int(level) if level else 0))
    lines = [l for l in r.stderr.splitlines() if l.startswith("[tdct ")]
    n = int(level) if level else 0
    assert all(int(l[6]) <= n for l in lines)  # nothing above the level
    has = lambda what: any(what in l for l in lines)
    assert has("error: a batch of 1 requests failed on the device (fake device") == (n >= 1)
    assert has("server create: continuous batching") == (n >= 2)
    assert has("server destroy: 6 submitted") == (n >= 2)
    assert has("server batch: ") == (n >= 3)
