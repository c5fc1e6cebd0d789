"""The batch form without allocation, tdct_batch_run_static, through the C
ABI: its outputs equal those of the same images run through tdct_batch_plan
+ tdct_batch_run, byte for byte (tolerance 0, padding included), on two
calls in a row on one stream whose second, smaller batch overwrites the
first's tables in the device array; and tables larger than the array are
refused before any device work."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import sync

pytestmark = pytest.mark.gpu

SENTINEL = 0xA7


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


class Batch:
    """Images of every op with uneven sizes and strides; inputs once, and
    one set of sentinel-filled outputs per run that is compared."""

    def __init__(self, tdct, sizes, seed):
        import torch
        rng = np.random.default_rng(seed)
        self.qtabs = [synth.qtable(1, s) for s in (1, 4)] + [rng.integers(1, 4096, 64).astype(np.uint16)]
        ops = [tdct.OP_ENCODE, tdct.OP_DECODE, tdct.OP_ROUNDTRIP, tdct.OP_ENCODE_I8ZZ, tdct.OP_FORWARD]
        self.items = []
        for k, (w, h) in enumerate(sizes):
            op = ops[(k + seed) % len(ops)]
            stride = w + 8 * (k % 3) + (3 if k % 5 == 2 else 0)
            img = synth.textured(w, h, 900 + 31 * seed + k, stride=stride)
            nblk = (w // 8) * (h // 8)
            it = dict(op=op, w=w, h=h, stride=stride, img=img, nblk=nblk, qt=k % len(self.qtabs),
                      keep=[64, 10, 25, 1][k % 4], src=torch.from_numpy(img).cuda())
            if op == tdct.OP_DECODE:
                it["qin"] = rng.integers(-2000, 2001, size=(nblk, 64)).astype(np.int16)
                it["cin"] = torch.from_numpy(it["qin"]).cuda()
            it["cbytes"] = nblk * 64 * {tdct.OP_ENCODE: 2, tdct.OP_ROUNDTRIP: 2, tdct.OP_ENCODE_I8ZZ: 1,
                                        tdct.OP_FORWARD: 4, tdct.OP_DECODE: 0}[op]
            self.items.append(it)
        self.tdct = tdct

    def outputs(self):
        """Fresh sentinel-filled output buffers and the descriptors naming them."""
        import torch
        t = self.tdct
        outs, descs = [], []
        for it in self.items:
            o = {"dst": torch.full((it["h"], it["stride"]), SENTINEL, dtype=torch.uint8, device="cuda")}
            if it["cbytes"]:
                o["coef"] = torch.full((it["cbytes"],), SENTINEL, dtype=torch.uint8, device="cuda")
            coef = it["cin"] if it["op"] == t.OP_DECODE else o.get("coef")
            descs.append(t.image_desc(it["op"], it["w"], it["h"], qtab=it["qt"], keep=it["keep"], src=it["src"],
                                      src_stride=it["stride"], coef=coef, dst=o["dst"], dst_stride=it["stride"]))
            outs.append(o)
        return outs, descs


def _host(outs):
    return [{k: v.cpu().numpy() for k, v in o.items()} for o in outs]


def _check_oracle(tdct, B, outs, every=3):
    for k, (it, o) in enumerate(zip(B.items, outs)):
        if k % every:
            continue
        op, w, h, Q = it["op"], it["w"], it["h"], B.qtabs[it["qt"]]
        if op == tdct.OP_ENCODE:
            assert np.array_equal(o["coef"].view(np.int16).reshape(-1, 64), O.quantise(it["img"], Q, it["keep"], w=w)), k
        elif op == tdct.OP_DECODE:
            assert np.array_equal(o["dst"][:, :w], O.inverse(it["qin"], Q, w, h)), k
        elif op == tdct.OP_ROUNDTRIP:
            q = O.quantise(it["img"], Q, it["keep"], w=w)
            assert np.array_equal(o["coef"].view(np.int16).reshape(-1, 64), q), k
            assert np.array_equal(o["dst"][:, :w], O.inverse(q, Q, w, h)), k
        elif op == tdct.OP_ENCODE_I8ZZ:
            assert np.array_equal(o["coef"].view(np.int8).reshape(-1, 64), O.quantise_i8_zigzag(it["img"], Q, w=w)), k
        else:
            assert np.array_equal(o["coef"].view(np.int32).reshape(-1, 64), O.forward(it["img"], w=w)), k


def _run_plan(tdct, B, descs, stream):
    plan = tdct.tdct_batch_plan(descs, B.qtabs)
    try:
        tdct.tdct_batch_run(plan, stream)
        sync()
    finally:
        tdct.tdct_plan_free(plan)


def _same(a, b):
    assert len(a) == len(b)
    for k, (x, y) in enumerate(zip(a, b)):
        assert x.keys() == y.keys()
        for key in x:
            assert np.array_equal(x[key], y[key]), (k, key)


BIG = [(2048, 1024), (1032, 520)] + [(8 * a, 8 * b) for a, b in
                                     np.random.default_rng(7).integers(1, 60, size=(40, 2))]
SMALL = [(136, 72), (8, 8), (520, 48), (64, 1024), (24, 16), (40, 40)]


@pytest.mark.parametrize("tune", [None, dict(waves_per_group=4, groups_per_cu=1, tile_waves=2, xcd_remap=1,
                                             pixel_cache=1)])
def test_two_calls_in_a_row_equal_plan_runs(tdct, tune):
    import torch
    stream = torch.cuda.current_stream()
    A, Bsm = Batch(tdct, BIG, 1), Batch(tdct, SMALL, 2)
    pa, da = A.outputs()
    pb, db = Bsm.outputs()
    _run_plan(tdct, A, da, stream)
    _run_plan(tdct, Bsm, db, stream)
    want_a, want_b = _host(pa), _host(pb)
    _check_oracle(tdct, A, want_a)
    _check_oracle(tdct, Bsm, want_b, every=1)
    sa, da2 = A.outputs()
    sb, db2 = Bsm.outputs()
    # back to back on one stream: the second call's tables overwrite the
    # first's only after the first kernel, in stream order
    tdct.tdct_batch_run_static(da2, A.qtabs, tune=tune, stream=stream)
    tdct.tdct_batch_run_static(db2, Bsm.qtabs, tune=tune, stream=stream)
    sync()
    _same(_host(sa), want_a)
    _same(_host(sb), want_b)
    # and the large batch again after the small one
    sa2, da3 = A.outputs()
    tdct.tdct_batch_run_static(da3, A.qtabs, tune=tune, stream=stream)
    sync()
    _same(_host(sa2), want_a)


def test_refusals_before_device_work(tdct):
    import torch
    L = tdct.lib()
    q = (tdct.tdct_qtable * 1)(tdct.qtable(np.ones(64)))
    src = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")

    def call(n):
        out = torch.full((n * 128,), SENTINEL, dtype=torch.uint8, device="cuda")
        base = out.data_ptr()
        descs = (tdct.tdct_image_desc * n)(*[tdct.image_desc(tdct.OP_ENCODE, 8, 8, src=src, src_stride=8,
                                                             coef=base + 128 * k) for k in range(n)])
        st = L.tdct_batch_run_static(descs, n, q, 1, None, ctypes.c_void_p(0))
        sync()
        assert (out.cpu().numpy() == SENTINEL).all()  # nothing was written
        return st

    # descriptors and constants alone exceed the array
    assert call(25000) == tdct.TDCT_ENOMEM
    # with the tiles they exceed it (checked once the device is known)
    assert call(20000) == tdct.TDCT_ENOMEM
    # an in-place round trip is refused like in a plan
    plane = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    d = tdct.image_desc(tdct.OP_ROUNDTRIP, 64, 64, src=plane, src_stride=64, dst=plane, dst_stride=64)
    assert L.tdct_batch_run_static((tdct.tdct_image_desc * 1)(d), 1, q, 1, None, None) == tdct.TDCT_EINVAL
    # an empty batch is a no-op
    assert L.tdct_batch_run_static(None, 0, q, 1, None, None) == tdct.TDCT_OK


def test_largest_batch_that_fits(tdct):
    """Close to the array's capacity: 18,000 single-block encodes (15.2 MB of
    tables) give the plan path's bytes."""
    import torch
    n = 18000
    img = synth.textured(8, 8 * n, 77)
    src = torch.from_numpy(img).cuda()
    Q = [synth.qtable(1, 5)]
    want = torch.full((n * 128,), SENTINEL, dtype=torch.uint8, device="cuda")
    got = torch.full_like(want, SENTINEL)

    def descs(out):
        b = out.data_ptr()
        return [tdct.image_desc(tdct.OP_ENCODE, 8, 8, keep=64, src=src.data_ptr() + 64 * k, src_stride=8,
                                coef=b + 128 * k) for k in range(n)]

    plan = tdct.tdct_batch_plan(descs(want), Q)
    try:
        tdct.tdct_batch_run(plan)
    finally:
        tdct.tdct_plan_free(plan)
    tdct.tdct_batch_run_static(descs(got), Q)
    sync()
    w, g = want.cpu().numpy(), got.cpu().numpy()
    assert np.array_equal(w, g)
    assert np.array_equal(w.view(np.int16).reshape(-1, 64), O.quantise(img, Q[0], 64))
