"""Serving form on the GPU: a Poisson mix of encode and decode requests of
uneven sizes, admitted under a budget and continuously batched over several
streams. Every request's output in the mix must be byte-identical to the
same request served alone (tolerance 0), sampled requests must equal the
oracle, and the arena must never exceed its budget."""
import ctypes
import os

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import sync

pytestmark = pytest.mark.gpu

POOL_SIDE = 1024


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


def _hip():
    import torch
    lib = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    lib.hipMemcpy.restype = ctypes.c_int
    return lib


def _read(hip, ptr, nbytes):
    out = np.empty(nbytes, np.uint8)
    assert hip.hipMemcpy(out.ctypes.data, ptr, nbytes, 2) == 0  # device -> host
    return out


class Workload:
    def __init__(self, tdct, rate=3000.0, seconds=0.12, seed=55):
        import torch
        rng = np.random.default_rng(seed)
        self.planes = [synth.textured(POOL_SIDE, POOL_SIDE, 7000 + k) for k in range(2)]
        self.coefs = [rng.integers(-300, 301, size=((POOL_SIDE // 8) ** 2, 64)).astype(np.int16)
                      for _ in range(2)]
        self.dplanes = [torch.from_numpy(p).cuda() for p in self.planes]
        self.dcoefs = [torch.from_numpy(c).cuda() for c in self.coefs]
        tr = synth.serving_trace(rate, seconds, seed=seed, lo=32, hi=POOL_SIDE)
        self.tr = tr
        self.reqs, self.meta = [], []
        for k in range(len(tr["t"])):
            w, h, s, op = int(tr["w"][k]), int(tr["h"][k]), int(tr["s"][k]), int(tr["op"][k])
            p = k % 2
            Q = synth.qtable(1, s)
            keep = 64 if k % 5 else 10
            if op == 0:
                r = tdct.request(tdct.OP_ENCODE, w, h, self.dplanes[p], Q, keep=keep, in_stride=POOL_SIDE)
                nbytes = w * h * 2
            else:
                r = tdct.request(tdct.OP_DECODE, w, h, self.dcoefs[p], Q)
                nbytes = w * h
            self.reqs.append(r)
            self.meta.append(dict(op=op, w=w, h=h, p=p, Q=Q, keep=keep, nbytes=nbytes))
        self.arrival = (tr["t"] * 1e6).tolist()

    def expected(self, k):
        m = self.meta[k]
        if m["op"] == 0:
            img = np.ascontiguousarray(self.planes[m["p"]][:m["h"], :m["w"]])
            return O.quantise(img, m["Q"], m["keep"]).view(np.uint8).reshape(-1)
        nblk = (m["w"] // 8) * (m["h"] // 8)
        return O.inverse(self.coefs[m["p"]][:nblk], m["Q"], m["w"], m["h"]).reshape(-1)


def _serve(tdct, W, cfg, idx=None, arrival=True):
    hip = _hip()
    srv = tdct.tdct_server_create(cfg)
    try:
        reqs = W.reqs if idx is None else [W.reqs[k] for k in idx]
        arr = W.arrival if (idx is None and arrival) else [0.0] * len(reqs)
        tickets, lat, st = tdct.tdct_server_replay(srv, reqs, arr, keep_outputs=True)
        outs = []
        for t, s_ in zip(tickets, st):
            assert s_ == tdct.TDCT_OK
            r = tdct.tdct_server_poll(srv, t)
            outs.append(_read(hip, r.output, r.output_bytes))
        stats = tdct.tdct_server_stats(srv)
        for t in tickets:
            tdct.tdct_server_release(srv, t)
        assert tdct.tdct_server_stats(srv)["arena_bytes_in_use"] == 0
        return outs, lat, stats
    finally:
        tdct.tdct_server_destroy(srv)


def test_mix_equals_alone_and_oracle(tdct):
    W = Workload(tdct, rate=10000.0, seconds=0.03)
    n = len(W.reqs)
    assert n > 100
    budget = 1 << 30
    cfg = tdct.server_cfg(budget, streams=4, max_batch=16, max_wait_us=300, batching=1)
    mix, lat, stats = _serve(tdct, W, cfg)
    assert stats["completed"] == n and stats["failed"] == 0
    assert stats["arena_high_water"] <= budget
    assert stats["mean_batch"] > 1.0  # requests really shared launches
    # alone: each request on its own, one at a time, through a fresh server
    alone_cfg = tdct.server_cfg(budget, streams=1, max_batch=1, batching=1)
    for k in range(n):
        out, _, _ = _serve(tdct, W, alone_cfg, idx=[k])
        assert np.array_equal(mix[k], out[0]), k
    # per-request plain launches give the same bytes too
    per, _, st2 = _serve(tdct, W, tdct.server_cfg(budget, streams=4, max_batch=1, batching=0))
    assert st2["mean_batch"] == 1.0
    for k in range(n):
        assert np.array_equal(mix[k], per[k]), k
    # oracle on a sample (and on every request that is small)
    rng = np.random.default_rng(1)
    sample = set(rng.choice(n, 40, replace=False).tolist()) | {k for k in range(n) if
                                                              W.meta[k]["w"] * W.meta[k]["h"] <= 64 * 64}
    for k in sorted(sample):
        assert np.array_equal(mix[k], W.expected(k)), k


def test_batches_take_tuned_shapes_from_the_cache(tdct, tmp_path):
    """A server created with tune_cache = 1 launches its batches in the shapes
    the autotune cache holds for their class: plans made of the same kind of
    requests are tuned first (storing entries), then the requests arrive at
    once; the cache is hit and every output equals one plain launch per
    request, and sampled outputs equal the oracle."""
    import torch
    W = Workload(tdct, rate=10000.0, seconds=0.03, seed=57)
    n = len(W.reqs)
    try:
        tdct.tdct_tune_cache_open(str(tmp_path / "tune.json"))
        keep_alive = []
        for lo, hi in ((0, 4), (0, 16), (16, 32)):
            descs, qtabs = [], []
            for k in range(lo, min(hi, n)):
                m = W.meta[k]
                qtabs.append(m["Q"])
                if m["op"] == 0:
                    out = torch.empty(m["w"] * m["h"] // 64 * 64, dtype=torch.int16, device="cuda")
                    descs.append(tdct.image_desc(tdct.OP_ENCODE, m["w"], m["h"], qtab=len(qtabs) - 1,
                                                 keep=m["keep"], src=W.dplanes[m["p"]], src_stride=POOL_SIDE,
                                                 coef=out))
                else:
                    out = torch.empty(m["w"] * m["h"], dtype=torch.uint8, device="cuda")
                    descs.append(tdct.image_desc(tdct.OP_DECODE, m["w"], m["h"], qtab=len(qtabs) - 1,
                                                 coef=W.dcoefs[m["p"]], dst=out, dst_stride=m["w"]))
                keep_alive.append(out)
            plan = tdct.tdct_batch_plan(descs, qtabs)
            try:
                tdct.tdct_autotune(plan, reps=1)
            finally:
                tdct.tdct_plan_free(plan)
        stored = tdct.tdct_tune_cache_info()
        assert stored["entries"] >= 1
        cfg = tdct.server_cfg(1 << 30, streams=2, max_batch=16, max_wait_us=0, batching=1, tune_cache=1)
        mix, _, stats = _serve(tdct, W, cfg, idx=list(range(n)))
        assert stats["failed"] == 0 and stats["mean_batch"] > 1.0
        assert tdct.tdct_tune_cache_info()["batch_hits"] > 0
    finally:
        tdct.tdct_tune_cache_open(None)
    per, _, _ = _serve(tdct, W, tdct.server_cfg(1 << 30, streams=4, max_batch=1, batching=0))
    for k in range(n):
        assert np.array_equal(mix[k], per[k]), k
    rng = np.random.default_rng(3)
    for k in sorted(rng.choice(n, 30, replace=False).tolist()):
        assert np.array_equal(mix[k], W.expected(k)), k


def test_tight_budget_queues_instead_of_failing(tdct):
    """A budget that holds only the largest output: requests wait in FIFO
    order for memory and all complete once earlier outputs are released."""
    W = Workload(tdct, rate=20000.0, seconds=0.01, seed=56)
    biggest = max(m["nbytes"] for m in W.meta)
    budget = (biggest + 255) // 256 * 256 + 256
    hip = _hip()
    srv = tdct.tdct_server_create(tdct.server_cfg(budget, streams=2, max_batch=8, batching=1))
    try:
        tickets = [tdct.tdct_server_submit(srv, r) for r in W.reqs]
        for k, t in enumerate(tickets):
            r = tdct.tdct_server_wait(srv, t)
            assert r.status == tdct.TDCT_OK
            assert np.array_equal(_read(hip, r.output, r.output_bytes), W.expected(k)), k
            tdct.tdct_server_release(srv, t)
        st = tdct.tdct_server_stats(srv)
        assert st["failed"] == 0 and st["arena_high_water"] <= budget
        # replay keeping every output cannot fit this budget: refused, not hung
        with pytest.raises(tdct.TdctError) as e:
            tdct.tdct_server_replay(srv, W.reqs, [0.0] * len(W.reqs), keep_outputs=True)
        assert e.value.status == tdct.TDCT_ENOMEM
    finally:
        tdct.tdct_server_destroy(srv)


def test_host_payloads_equal_device_resident_results(tdct):
    """host_io requests: pinned host input, copied in, coded, copied back to a
    pinned host buffer; the bytes equal the device-resident path and the oracle."""
    import torch
    W = Workload(tdct, rate=10000.0, seconds=0.01, seed=57)
    n = len(W.reqs)
    hplanes = [torch.from_numpy(p).pin_memory() for p in W.planes]
    hcoefs = [torch.from_numpy(c).pin_memory() for c in W.coefs]
    outs, reqs = [], []
    for k, m in enumerate(W.meta):
        o = torch.zeros(m["nbytes"], dtype=torch.uint8).pin_memory()
        outs.append(o)
        if m["op"] == 0:
            reqs.append(tdct.request(tdct.OP_ENCODE, m["w"], m["h"], hplanes[m["p"]].data_ptr(), m["Q"],
                                     keep=m["keep"], in_stride=POOL_SIDE, host_output=o.data_ptr()))
        else:
            reqs.append(tdct.request(tdct.OP_DECODE, m["w"], m["h"], hcoefs[m["p"]].data_ptr(), m["Q"],
                                     host_output=o.data_ptr()))
    srv = tdct.tdct_server_create(tdct.server_cfg(64 << 20, streams=4, max_batch=16, max_wait_us=200))
    try:
        tickets, lat, st = tdct.tdct_server_replay(srv, reqs, W.arrival)
        assert all(s_ == tdct.TDCT_OK for s_ in st)
        stats = tdct.tdct_server_stats(srv)
        assert stats["arena_bytes_in_use"] == 0  # staging and outputs went back
    finally:
        tdct.tdct_server_destroy(srv)
    dev, _, _ = _serve(tdct, W, tdct.server_cfg(1 << 30, streams=4, max_batch=16, batching=1))
    for k in range(n):
        assert np.array_equal(outs[k].numpy(), dev[k]), k
    for k in range(0, n, 7):
        assert np.array_equal(outs[k].numpy(), W.expected(k)), k


# ---- resident mode -----------------------------------------------------------
# Small queue and tile ring, so that both wrap many times during the mix.
RESIDENT = dict(resident=1, resident_jobs=16, resident_tiles=1024, resident_idle_us=5000)


def test_resident_mix_equals_stream_mode_and_oracle(tdct):
    W = Workload(tdct, rate=10000.0, seconds=0.03, seed=58)
    n = len(W.reqs)
    assert n > 100
    budget = 1 << 30
    res, lat, st = _serve(tdct, W, tdct.server_cfg(budget, **RESIDENT))
    assert st["completed"] == n and st["failed"] == 0
    assert st["batches"] >= 1 and st["arena_high_water"] <= budget
    per, _, _ = _serve(tdct, W, tdct.server_cfg(budget, streams=4, max_batch=1, batching=0))
    for k in range(n):
        assert np.array_equal(res[k], per[k]), k
    rng = np.random.default_rng(2)
    for k in sorted(set(rng.choice(n, 30, replace=False).tolist())):
        assert np.array_equal(res[k], W.expected(k)), k


def test_resident_sees_inputs_rewritten_between_requests(tdct):
    """The resident kernel reads each request's inputs as they are when the
    request is submitted, also where an earlier request read the same buffer
    (so its XCD's L2 may hold the old bytes) and the kernel has kept running
    since. One buffer of pixels and one of coefficients are rewritten before
    every request; every output must equal the oracle on the new content."""
    import torch
    hip = _hip()
    side = 1024
    rng = np.random.default_rng(77)
    X = torch.empty((side, side), dtype=torch.uint8, device="cuda")
    C = torch.empty(((side // 8) ** 2, 64), dtype=torch.int16, device="cuda")
    srv = tdct.tdct_server_create(tdct.server_cfg(1 << 30, resident=1, resident_idle_us=500000))
    got, cases = [], []
    try:
        inputs = [(synth.textured(side, side, 9000 + k),
                   rng.integers(-400, 401, size=((side // 8) ** 2, 64)).astype(np.int16)) for k in range(24)]
        for k, (img, coefs) in enumerate(inputs):
            X.copy_(torch.from_numpy(img))
            C.copy_(torch.from_numpy(coefs))
            # the copies' own stream only: a device-wide synchronize would wait
            # for the resident kernel to go idle and exit
            torch.cuda.current_stream().synchronize()
            w, h = [(1024, 1024), (512, 1024), (1024, 256), (776, 520)][k % 4]
            Q = synth.qtable(1, 1 + k % 8)
            te = tdct.tdct_server_submit(srv, tdct.request(tdct.OP_ENCODE, w, h, X, Q, in_stride=side))
            td = tdct.tdct_server_submit(srv, tdct.request(tdct.OP_DECODE, w, h, C, Q))
            re, rd = tdct.tdct_server_wait(srv, te), tdct.tdct_server_wait(srv, td)
            assert re.status == tdct.TDCT_OK and rd.status == tdct.TDCT_OK
            got.append((_read(hip, re.output, re.output_bytes), _read(hip, rd.output, rd.output_bytes)))
            cases.append((w, h, Q))
            tdct.tdct_server_release(srv, te)
            tdct.tdct_server_release(srv, td)
        # the kernel stayed up across requests (it lives one second at a time)
        assert tdct.tdct_server_stats(srv)["batches"] <= 2
    finally:
        tdct.tdct_server_destroy(srv)
    for k, ((img, coefs), (w, h, Q), (ge, gd)) in enumerate(zip(inputs, cases, got)):
        want_e = O.quantise(np.ascontiguousarray(img[:h, :w]), Q, 64).view(np.uint8).reshape(-1)
        want_d = O.inverse(coefs[:(w // 8) * (h // 8)], Q, w, h).reshape(-1)
        assert np.array_equal(ge, want_e), (k, "encode")
        assert np.array_equal(gd, want_d), (k, "decode")


def test_resident_single_worker_and_wrap(tdct):
    """One worker wave claims every tile; 4 queue slots and 256 tile slots."""
    W = Workload(tdct, rate=20000.0, seconds=0.005, seed=59)
    cfg = tdct.server_cfg(1 << 30, resident=1, resident_workers=1, resident_jobs=4,
                          resident_tiles=256, resident_idle_us=5000)
    res, _, st = _serve(tdct, W, cfg, arrival=False)
    assert st["completed"] == len(W.reqs) and st["failed"] == 0
    for k in range(len(W.reqs)):
        assert np.array_equal(res[k], W.expected(k)), k


def test_resident_kernel_relaunches_after_idle_exit(tdct):
    import time
    import torch
    hip = _hip()
    img = synth.textured(256, 128, 9)
    dimg = torch.from_numpy(img).cuda()
    Q = synth.qtable(1, 3)
    srv = tdct.tdct_server_create(tdct.server_cfg(1 << 24, resident=1, resident_idle_us=2000,
                                                  resident_workers=4))
    try:
        for _ in range(2):
            t = tdct.tdct_server_submit(srv, tdct.request(tdct.OP_ENCODE, 256, 128, dimg, Q, keep=20))
            r = tdct.tdct_server_wait(srv, t)
            assert r.status == tdct.TDCT_OK
            got = _read(hip, r.output, r.output_bytes)
            assert np.array_equal(got, O.quantise(img, Q, 20).view(np.uint8).reshape(-1))
            tdct.tdct_server_release(srv, t)
            time.sleep(0.05)  # past the idle limit: the kernel exits
        assert tdct.tdct_server_stats(srv)["batches"] == 2
        assert tdct.tdct_server_last_error(srv) == ""
    finally:
        tdct.tdct_server_destroy(srv)


def test_resident_large_and_ragged_requests(tdct):
    """Requests big enough for multi-tile work items on few workers (so the
    in-item prefetch runs), with odd block counts per row and partial last
    tiles, encode and decode, each equal to the oracle in full."""
    import torch
    hip = _hip()
    rng = np.random.default_rng(60)
    cases = []
    for k, (w, h) in enumerate([(4104, 1032), (2048, 2056), (1032, 4104), (3000, 8)]):
        img = synth.textured(w, h, 8000 + k)
        Q = synth.qtable(1, 1 + k)
        nblk = (w // 8) * (h // 8)
        coefs = rng.integers(-2000, 2001, size=(nblk, 64)).astype(np.int16)
        cases.append((w, h, img, Q, coefs, torch.from_numpy(img).cuda(), torch.from_numpy(coefs).cuda()))
    for workers in (3, 16, 40):  # 2, 16 and 32 ticket queues, unevenly staffed at 3 and 40
        srv = tdct.tdct_server_create(tdct.server_cfg(1 << 30, resident=1, resident_workers=workers,
                                                      resident_idle_us=5000))
        try:
            tickets = []
            for w, h, img, Q, coefs, dimg, dcoef in cases:
                tickets.append(tdct.tdct_server_submit(srv, tdct.request(tdct.OP_ENCODE, w, h, dimg, Q, keep=40)))
                tickets.append(tdct.tdct_server_submit(srv, tdct.request(tdct.OP_DECODE, w, h, dcoef, Q)))
            for k, (w, h, img, Q, coefs, _, _) in enumerate(cases):
                r = tdct.tdct_server_wait(srv, tickets[2 * k])
                assert r.status == tdct.TDCT_OK
                got = _read(hip, r.output, r.output_bytes).view(np.int16).reshape(-1, 64)
                assert np.array_equal(got, O.quantise(img, Q, 40, threads=8)), (workers, w, h, "encode")
                r = tdct.tdct_server_wait(srv, tickets[2 * k + 1])
                assert r.status == tdct.TDCT_OK
                got = _read(hip, r.output, r.output_bytes).reshape(h, w)
                assert np.array_equal(got, O.inverse(coefs, Q, w, h, threads=8)), (workers, w, h, "decode")
            assert tdct.tdct_server_last_error(srv) == ""
        finally:
            tdct.tdct_server_destroy(srv)


def test_resident_unaligned_encode_inputs(tdct):
    """Encode requests whose pixel rows are not 8-byte aligned (an odd start
    address, an odd stride) take the resident kernel's byte-wise coherent
    loads; every output equals the oracle in full, next to an aligned request
    served by the same launch."""
    import torch
    hip = _hip()
    side, stride = 1032, 1037
    img = synth.textured(side, side, 9100)
    host = np.zeros(side * stride + 64, np.uint8)
    base = 3
    for y in range(side):
        host[base + y * stride: base + y * stride + side] = img[y]
    dbuf = torch.from_numpy(host).cuda()
    aligned = torch.from_numpy(img).cuda()
    # (w, h, byte offset of the window's first pixel inside the plane)
    cases = [(1032, 1032, 0), (520, 776, 1 + 5 * stride), (8, 8, 7 + stride), (1024, 16, 5)]
    srv = tdct.tdct_server_create(tdct.server_cfg(1 << 30, resident=1, resident_workers=64,
                                                  resident_idle_us=5000))
    try:
        tickets = []
        for k, (w, h, off) in enumerate(cases):
            Q = synth.qtable(1, 1 + k)
            tickets.append(tdct.tdct_server_submit(srv, tdct.request(
                tdct.OP_ENCODE, w, h, dbuf.data_ptr() + base + off, Q, keep=48, in_stride=stride)))
        ta = tdct.tdct_server_submit(srv, tdct.request(tdct.OP_ENCODE, side, side, aligned,
                                                       synth.qtable(1, 2), keep=48, in_stride=side))
        for k, (w, h, off) in enumerate(cases):
            r = tdct.tdct_server_wait(srv, tickets[k])
            assert r.status == tdct.TDCT_OK
            got = _read(hip, r.output, r.output_bytes).view(np.int16).reshape(-1, 64)
            y0, x0 = divmod(off, stride)
            window = np.ascontiguousarray(img[y0:y0 + h, x0:x0 + w])
            assert np.array_equal(got, O.quantise(window, synth.qtable(1, 1 + k), 48, threads=8)), (w, h, off)
        r = tdct.tdct_server_wait(srv, ta)
        assert r.status == tdct.TDCT_OK
        got = _read(hip, r.output, r.output_bytes).view(np.int16).reshape(-1, 64)
        assert np.array_equal(got, O.quantise(img, synth.qtable(1, 2), 48, threads=8))
        assert tdct.tdct_server_last_error(srv) == ""
    finally:
        tdct.tdct_server_destroy(srv)


# ---- the serving workload at its own request sizes ---------------------------
# Sides log-uniform multiples of 8 in [32, 8192] with aspect <= 4, encode and
# decode with p = 1/2, s in {1..8}, payloads windows of 8192^2 planes; plus
# requests of 32 Mpx and more, so that batches are cut at max_batch_px. Every
# output is compared with the oracle in full, on the host threads.
CFG5_SIDE = 8192
CFG5_THREADS = 16


class Cfg5Workload:
    def __init__(self, tdct, rate=1000.0, seconds=0.12, seed=61):
        import torch
        self.planes = [synth.plane(CFG5_SIDE, CFG5_SIDE, 5100 + k) for k in range(2)]
        # decode inputs: the oracle's encoding of each plane under its own table
        self.qin = [synth.qtable(1, 2 + 3 * k) for k in range(2)]
        self.coefs = [O.quantise(p, q, 64, threads=CFG5_THREADS) for p, q in zip(self.planes, self.qin)]
        self.dplanes = [torch.from_numpy(p).cuda() for p in self.planes]
        self.dcoefs = [torch.from_numpy(c).cuda() for c in self.coefs]
        tr = synth.serving_trace(rate, seconds, seed=seed, lo=32, hi=CFG5_SIDE)
        ops = [int(x) for x in tr["op"]]
        sides = [(int(w), int(h)) for w, h in zip(tr["w"], tr["h"])]
        scales = [int(s) for s in tr["s"]]
        # requests of 32 Mpx and more (the largest the workload draws), one of each op
        for k, (w, h) in enumerate([(8192, 8192), (8192, 4096), (6144, 6144), (4096, 8192)]):
            at = (k + 1) * len(ops) // 5
            ops.insert(at, k % 2)
            sides.insert(at, (w, h))
            scales.insert(at, 1 + 2 * k)
        self.reqs, self.meta = [], []
        for k, (op, (w, h), s) in enumerate(zip(ops, sides, scales)):
            p, Q = k % 2, synth.qtable(1, s)
            keep = 64 if k % 7 else 10
            if op == 0:
                r = tdct.request(tdct.OP_ENCODE, w, h, self.dplanes[p], Q, keep=keep, in_stride=CFG5_SIDE)
            else:
                r = tdct.request(tdct.OP_DECODE, w, h, self.dcoefs[p], Q)
            self.reqs.append(r)
            self.meta.append(dict(op=op, w=w, h=h, p=p, Q=Q, keep=keep))
        t = np.sort(np.random.default_rng(seed).uniform(0, seconds * 1e6, len(self.reqs)))
        self.arrival = t.tolist()

    def expected(self, k):
        m = self.meta[k]
        w, h = m["w"], m["h"]
        if m["op"] == 0:
            q = O.quantise(self.planes[m["p"]][:h], m["Q"], m["keep"], w=w, threads=CFG5_THREADS)
            return q.view(np.uint8).reshape(-1)
        nblk = (w // 8) * (h // 8)
        return O.inverse(self.coefs[m["p"]][:nblk], m["Q"], w, h, threads=CFG5_THREADS).reshape(-1)


@pytest.fixture(scope="module")
def cfg5(tdct):
    return Cfg5Workload(tdct)


def _check_all(W, outs, what):
    for k in range(len(W.reqs)):
        assert np.array_equal(outs[k], W.expected(k)), (what, k, W.meta[k]["w"], W.meta[k]["h"])


def test_cfg5_sizes_batched_stream_mode_against_oracle(tdct, cfg5):
    """Continuous batching over 4 streams at the serving workload's own sizes,
    arriving over 0.12 s, with a 16 Mpx batch cap: every output, the
    requests of 32 to 64 Mpx included, equals the oracle."""
    W = cfg5
    big = [k for k, m in enumerate(W.meta) if m["w"] * m["h"] >= 32 << 20]
    assert len(big) >= 4 and max(m["w"] for m in W.meta) == CFG5_SIDE
    budget = 8 << 30
    cfg = tdct.server_cfg(budget, streams=4, max_batch=64, batching=1, max_batch_px=16 << 20,
                          tune=dict(pixel_cache=1))
    outs, lat, st = _serve(tdct, W, cfg)
    assert st["completed"] == len(W.reqs) and st["failed"] == 0
    assert st["arena_high_water"] <= budget
    _check_all(W, outs, "batched")


def test_cfg5_sizes_burst_splits_batches_at_the_pixel_cap(tdct, cfg5):
    """The same requests all at once: batches form and are cut at the 16 Mpx
    cap (a large request rides alone or with a few small ones), under a budget
    that makes later requests wait for memory; every output equals the
    oracle, and equals one plain launch per request."""
    W = cfg5
    sizes = [m["w"] * m["h"] * (2 if m["op"] == 0 else 1) for m in W.meta]
    budget = (max(max(sizes) + 256, sum(sizes) // 3) + 255) // 256 * 256
    cfg = tdct.server_cfg(budget, streams=4, max_batch=64, batching=1, max_batch_px=16 << 20)
    hip = _hip()
    srv = tdct.tdct_server_create(cfg)
    try:
        tickets = [tdct.tdct_server_submit(srv, r) for r in W.reqs]
        res = []
        for k, t in enumerate(tickets):
            r = tdct.tdct_server_wait(srv, t)
            assert r.status == tdct.TDCT_OK, k
            res.append(r.batch_size)
            if W.meta[k]["w"] * W.meta[k]["h"] > 16 << 20:
                assert r.batch_size == 1, k  # above the cap: launched alone
            got = _read(hip, r.output, r.output_bytes)
            assert np.array_equal(got, W.expected(k)), ("burst", k)
            tdct.tdct_server_release(srv, t)
        st = tdct.tdct_server_stats(srv)
        assert st["failed"] == 0 and st["arena_high_water"] <= budget
        assert st["mean_batch"] > 1.0
    finally:
        tdct.tdct_server_destroy(srv)
    per, _, st2 = _serve(tdct, W, tdct.server_cfg(8 << 30, streams=4, max_batch=1, batching=0), arrival=False)
    assert st2["mean_batch"] == 1.0
    _check_all(W, per, "per-request")
