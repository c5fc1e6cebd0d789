"""Batch form on the GPU: one persistent launch over many images of uneven
sizes, its hipGraph replay, every launch shape the autotuner may pick, and
one plain launch per image must all give the oracle's bytes. The full-size
workloads run in the launch configuration the benchmark times: the 64 images
of 4096 x 4096 and the 10,000 ragged images are compared with the oracle in
full (every image, on the host threads), and so are all 256 4:2:0 frames."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import sync

pytestmark = pytest.mark.gpu

HOST_THREADS = 16


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


def _block(img, w, b):
    nbx = w // 8
    by, bx = divmod(int(b), nbx)
    return np.ascontiguousarray(img[8 * by:8 * by + 8, 8 * bx:8 * bx + 8])


class Ragged:
    """A mixed batch: every op, uneven sizes (odd blocks per row, strips,
    single blocks), strides wider than the image, several Q tables."""

    def __init__(self, tdct, seed=5, big=False):
        import torch
        rng = np.random.default_rng(seed)
        self.qtabs = [synth.qtable(1, s) for s in (1, 3, 8)] + [rng.integers(1, 4096, 64).astype(np.uint16)]
        sizes = [(8, 8), (24, 16), (136, 72), (1024, 64), (8, 1024), (520, 48), (40, 40), (2048, 24)]
        sizes += [(8 * int(a), 8 * int(b)) for a, b in rng.integers(1, 40, size=(24, 2))]
        if big:  # enough blocks for 128-block encoder tiles (a small plan uses 64)
            sizes = [(4096, 2048)] + sizes
        self.items = []
        ops = [tdct.OP_ENCODE, tdct.OP_DECODE, tdct.OP_ROUNDTRIP, tdct.OP_ENCODE_I8ZZ, tdct.OP_FORWARD]
        self.keep_alive = []
        for k, (w, h) in enumerate(sizes):
            op = ops[(k + seed) % len(ops)]
            stride = w + (8 * (k % 3)) + (3 if k % 7 == 3 else 0)
            img = synth.textured(w, h, 500 + k, stride=stride)
            qt = k % len(self.qtabs)
            keep = [64, 10, 25, 1][k % 4]
            nblk = (w // 8) * (h // 8)
            it = dict(op=op, w=w, h=h, img=img, qt=qt, keep=keep, stride=stride, nblk=nblk)
            it["src"] = torch.from_numpy(img).cuda()
            if op == tdct.OP_DECODE:
                qin = rng.integers(-2000, 2000, size=(nblk, 64)).astype(np.int16)
                it["qin"] = qin
                it["coef"] = torch.from_numpy(qin).cuda()
            elif op in (tdct.OP_ENCODE, tdct.OP_ROUNDTRIP):
                it["coef"] = torch.zeros((nblk, 64), dtype=torch.int16, device="cuda")
            elif op == tdct.OP_ENCODE_I8ZZ:
                it["coef"] = torch.zeros((nblk, 64), dtype=torch.int8, device="cuda")
            else:
                it["coef"] = torch.zeros((nblk, 64), dtype=torch.int32, device="cuda")
            it["dst"] = torch.zeros((h, stride), dtype=torch.uint8, device="cuda")
            self.items.append(it)
        self.descs = []
        for it in self.items:
            self.descs.append(tdct.image_desc(it["op"], it["w"], it["h"], qtab=it["qt"], keep=it["keep"],
                                              src=it["src"], src_stride=it["stride"], coef=it["coef"],
                                              dst=it["dst"], dst_stride=it["stride"]))

    def clear(self):
        for it in self.items:
            if it["op"] != 1:
                it["coef"].zero_()
            it["dst"].zero_()

    def check(self, tdct):
        sync()
        for it in self.items:
            op, w, h, Q = it["op"], it["w"], it["h"], self.qtabs[it["qt"]]
            img = it["img"]
            if op == tdct.OP_ENCODE:
                assert np.array_equal(it["coef"].cpu().numpy(), O.quantise(img, Q, it["keep"], w=w))
            elif op == tdct.OP_DECODE:
                assert np.array_equal(it["dst"].cpu().numpy()[:, :w], O.inverse(it["qin"], Q, w, h))
            elif op == tdct.OP_ROUNDTRIP:
                q = O.quantise(img, Q, it["keep"], w=w)
                assert np.array_equal(it["coef"].cpu().numpy(), q)
                assert np.array_equal(it["dst"].cpu().numpy()[:, :w], O.inverse(q, Q, w, h))
            elif op == tdct.OP_ENCODE_I8ZZ:
                assert np.array_equal(it["coef"].cpu().numpy(), O.quantise_i8_zigzag(img, Q, w=w))
            else:
                assert np.array_equal(it["coef"].cpu().numpy(), O.forward(img, w=w))


def test_ragged_mixed_batch_one_launch(tdct):
    R = Ragged(tdct)
    plan = tdct.tdct_batch_plan(R.descs, R.qtabs)
    try:
        info = tdct.tdct_plan_info_get(plan)
        assert info["images"] == len(R.items)
        assert info["blocks"] == sum(it["nblk"] for it in R.items)
        tdct.tdct_batch_run(plan)
        R.check(tdct)
    finally:
        tdct.tdct_plan_free(plan)


def test_tile_size_and_default_shape_of_plans(tdct):
    """Tiles are 128 blocks for encoder-side ops and 64 for the decoder and
    the int32 forward, except that a plan whose 128-block tiles would number
    fewer than the device's SIMDs cuts encoder-side work into 64-block
    tiles; the default launch shape is one wave per workgroup over a full
    grid. (Descriptors only: nothing is launched.)"""
    import torch
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    fake = 0x100000
    out = 1 << 40  # outputs apart from inputs: a plan refuses overlapping ones
    q = [np.ones(64, np.uint16)]

    def tiles(descs):
        plan = tdct.tdct_batch_plan(descs, q)
        try:
            info = tdct.tdct_plan_info_get(plan)
        finally:
            tdct.tdct_plan_free(plan)
        assert info["tune"] == {"waves_per_group": 1, "groups_per_cu": 4096, "tile_waves": 1,
                                "xcd_remap": 0, "pixel_cache": 0}
        return info["tiles"]

    def enc(side):
        return tdct.image_desc(tdct.OP_ENCODE, side, side, src=fake, src_stride=side, coef=out)

    def dec(side):
        return tdct.image_desc(tdct.OP_DECODE, side, side, coef=fake, dst=out, dst_stride=side)

    def fwd(side):
        return tdct.image_desc(tdct.OP_FORWARD, side, side, src=fake, src_stride=side, coef=out)

    small = (512 // 8) ** 2  # 4096 blocks: 32 encoder tiles of 128
    assert small // 128 < simds
    assert tiles([enc(512)]) == small // 64
    assert tiles([dec(512)]) == small // 64
    assert tiles([enc(512), dec(512)]) == 2 * small // 64
    big = (4096 // 8) ** 2  # 262144 blocks per image
    assert 16 * big // 128 >= simds
    assert tiles([enc(4096)] * 16) == 16 * big // 128
    assert tiles([enc(4096)] * 16 + [dec(512)]) == 16 * big // 128 + small // 64
    assert tiles([fwd(4096)] * 16) == 16 * big // 64


def test_empty_plan_is_a_no_op(tdct):
    plan = tdct.tdct_batch_plan([], [np.ones(64, np.uint16)])
    try:
        info = tdct.tdct_plan_info_get(plan)
        assert info["images"] == 0 and info["tiles"] == 0 and info["blocks"] == 0
        tdct.tdct_batch_run(plan)
        tdct.tdct_batch_graph(plan)
        assert tdct.tdct_autotune(plan, reps=1) == info["tune"]
        tdct.tdct_run_per_image([], [np.ones(64, np.uint16)])
        sync()
    finally:
        tdct.tdct_plan_free(plan)


def test_graph_replays_equal_direct_launch(tdct):
    R = Ragged(tdct, seed=6)
    plan = tdct.tdct_batch_plan(R.descs, R.qtabs)
    try:
        for _ in range(3):
            R.clear()
            sync()
            tdct.tdct_batch_graph(plan)
            R.check(tdct)
    finally:
        tdct.tdct_plan_free(plan)


@pytest.mark.parametrize("tune", [dict(waves_per_group=1, groups_per_cu=1, tile_waves=1),
                                  dict(waves_per_group=2, groups_per_cu=3, tile_waves=2),
                                  dict(waves_per_group=8, groups_per_cu=4, tile_waves=4),
                                  dict(waves_per_group=8, groups_per_cu=4096, tile_waves=1),
                                  dict(waves_per_group=1, groups_per_cu=4096, tile_waves=2),
                                  dict(waves_per_group=1, groups_per_cu=4096, tile_waves=1, xcd_remap=1),
                                  dict(waves_per_group=4, groups_per_cu=1, tile_waves=2, xcd_remap=1),
                                  dict(waves_per_group=2, groups_per_cu=3, tile_waves=4, xcd_remap=1),
                                  dict(waves_per_group=1, groups_per_cu=4096, tile_waves=1, xcd_remap=1,
                                       pixel_cache=1),
                                  dict(waves_per_group=4, groups_per_cu=2, tile_waves=2, pixel_cache=1)])
def test_every_launch_shape_gives_same_bytes(tdct, tune):
    R = Ragged(tdct, seed=7)
    plan = tdct.tdct_batch_plan(R.descs, R.qtabs, tune=tune)
    try:
        tdct.tdct_batch_run(plan)
        R.check(tdct)
    finally:
        tdct.tdct_plan_free(plan)


@pytest.mark.parametrize("seed", range(24))
def test_random_plans_and_launch_shapes(tdct, seed):
    """Seeded mixed plans (every op, uneven sizes and strides; odd seeds add
    a 4096 x 2048 image, which makes the plan large enough for 128-block
    encoder tiles) in a random launch shape, XCD order and pixel cache
    policy included, against the oracle."""
    rng = np.random.default_rng(9000 + seed)
    tune = dict(waves_per_group=int(rng.choice([1, 2, 4, 8])),
                groups_per_cu=int(rng.choice([1, 2, 3, 4, 8, 16, 4096])),
                tile_waves=int(rng.choice([1, 2, 4])), xcd_remap=int(rng.integers(2)),
                pixel_cache=int(rng.integers(2)))
    print("seed", seed, "tune", tune, flush=True)
    R = Ragged(tdct, seed=100 + seed, big=seed % 2 == 1)
    plan = tdct.tdct_batch_plan(R.descs, R.qtabs, tune=tune)
    try:
        assert tdct.tdct_plan_info_get(plan)["tune"] == tune
        tdct.tdct_batch_run(plan)
        R.check(tdct)
    finally:
        tdct.tdct_plan_free(plan)


def test_autotuner_result_and_per_image_launches(tdct):
    R = Ragged(tdct, seed=8)
    plan = tdct.tdct_batch_plan(R.descs, R.qtabs)
    try:
        best = tdct.tdct_autotune(plan, reps=1)
        assert best["waves_per_group"] in (1, 2, 4, 8) and best["xcd_remap"] in (0, 1)
        assert best["pixel_cache"] in (0, 1)
        assert tdct.tdct_plan_info_get(plan)["tune"] == best  # the plan keeps the winner
        R.clear()
        tdct.tdct_batch_run(plan)
        R.check(tdct)
        R.clear()
        tdct.tdct_run_per_image(R.descs, R.qtabs)
        R.check(tdct)
    finally:
        tdct.tdct_plan_free(plan)


def test_autotune_cache_skips_the_search_and_keeps_the_shape(tdct, tmp_path):
    """With the autotune cache on, the first autotune of a class times
    candidates and stores the winner in the file; a new process (here: the
    file opened again) applies the stored shape to another plan of the same
    class without timing anything, and that plan's outputs are the oracle's.
    A plan of another class misses; its store keeps an entry another process
    wrote to the file in the meantime."""
    import time
    path = str(tmp_path / "tune.json")
    try:
        tdct.tdct_tune_cache_open(path)
        A = Ragged(tdct, seed=21)
        pa = tdct.tdct_batch_plan(A.descs, A.qtabs)
        try:
            best = tdct.tdct_autotune(pa, reps=1)
        finally:
            tdct.tdct_plan_free(pa)
        info = tdct.tdct_tune_cache_info()
        assert info["stores"] == 1 and info["entries"] == 1 and info["misses"] == 1
        text = open(path).read()
        assert '"format": "tdct-autotune-1"' in text and "/ops=" in text
        tdct.tdct_tune_cache_open(path)  # as a later process would
        B = Ragged(tdct, seed=21)  # same sizes and ops, new buffers
        pb = tdct.tdct_batch_plan(B.descs, B.qtabs)
        try:
            t0 = time.perf_counter()
            again = tdct.tdct_autotune(pb, reps=1)
            assert time.perf_counter() - t0 < 0.05  # no candidate was timed
            assert again == best and tdct.tdct_plan_info_get(pb)["tune"] == best
            tdct.tdct_batch_run(pb)
            B.check(tdct)
        finally:
            tdct.tdct_plan_free(pb)
        info = tdct.tdct_tune_cache_info()
        assert info["hits"] == 1 and info["stores"] == 0
        # another process stores a class in the file meanwhile: kept by the
        # next rewrite
        import json
        doc = json.load(open(path))
        other = "gfx950/src=00000000ffffffff/ops=4/tiles=3/aligned=0"
        doc["entries"][other] = [1, 4096, 1, 0, 0]
        json.dump(doc, open(path, "w"))
        C = Ragged(tdct, seed=22, big=True)  # more tiles: another size class
        pc = tdct.tdct_batch_plan(C.descs, C.qtabs)
        try:
            tdct.tdct_autotune(pc, reps=1)
            tdct.tdct_batch_run(pc)
            C.check(tdct)
        finally:
            tdct.tdct_plan_free(pc)
        info = tdct.tdct_tune_cache_info()
        assert info["stores"] == 1 and info["entries"] == 3 and info["write_errors"] == 0
        assert json.load(open(path))["entries"][other] == [1, 4096, 1, 0, 0]
        assert len(json.load(open(path))["entries"]) == 3
    finally:
        tdct.tdct_tune_cache_open(None)


# ---- full-size workloads ------------------------------------------------------

@pytest.mark.parametrize("tune", [None,
                                  dict(waves_per_group=1, groups_per_cu=4096, tile_waves=1, xcd_remap=1),
                                  dict(waves_per_group=4, groups_per_cu=1, tile_waves=2, xcd_remap=1),
                                  dict(waves_per_group=2, groups_per_cu=4096, tile_waves=1, xcd_remap=1,
                                       pixel_cache=1)])
def test_large_batch_64_images_4096(tdct, tune):
    """64 images of 4096 x 4096, per-image Q = 1 + s (i + j): one persistent
    encode launch and one decode launch, as timed by the benchmark, in the
    default launch shape, in the XCD-remapped shapes the autotuner picks for
    them and with cached pixel accesses."""
    import torch
    sizes, seeds, qs = synth.large_batch_spec()
    n, side = len(sizes), sizes[0][0]
    buf, off, strides = synth.batch(sizes, seeds)
    src = torch.from_numpy(buf).cuda()
    nblk = (side // 8) ** 2
    coef = torch.empty((n, nblk, 64), dtype=torch.int16, device="cuda")
    dst = torch.empty((n, side, side), dtype=torch.uint8, device="cuda")
    base = src.data_ptr()
    enc = [tdct.image_desc(tdct.OP_ENCODE, side, side, qtab=i, keep=64, src=base + int(off[i]),
                           src_stride=side, coef=coef[i]) for i in range(n)]
    dec = [tdct.image_desc(tdct.OP_DECODE, side, side, qtab=i, coef=coef[i], dst=dst[i],
                           dst_stride=side) for i in range(n)]
    pe, pd = tdct.tdct_batch_plan(enc, qs, tune=tune), tdct.tdct_batch_plan(dec, qs, tune=tune)
    try:
        tdct.tdct_batch_run(pe)
        tdct.tdct_batch_run(pd)
        sync()
        # every image in full: the oracle runs per image on the host threads
        ch, dh = coef.cpu().numpy(), dst.cpu().numpy()

        def check(i):
            img = synth.batch_view(buf, off, strides, sizes, i)
            q_ref, rec_ref = O.roundtrip(img, qs[i])
            return bool(np.array_equal(ch[i], q_ref) and np.array_equal(dh[i], rec_ref))

        with ThreadPoolExecutor(HOST_THREADS) as ex:
            ok = list(ex.map(check, range(n)))
        assert all(ok), [i for i, g in enumerate(ok) if not g]
        # any-size property: decoding an encoding at Q = 1 + s (i + j) never
        # moves a pixel of these fields by more than the quantiser allows
        assert int((dst.float() - src[:n * side * side].view(n, side, side).float()).abs().max()) < 128
    finally:
        tdct.tdct_plan_free(pe)
        tdct.tdct_plan_free(pd)


@pytest.mark.parametrize("tune", [dict(waves_per_group=8, groups_per_cu=4096, tile_waves=2),
                                  dict(waves_per_group=4, groups_per_cu=4096, tile_waves=1),
                                  dict(waves_per_group=4, groups_per_cu=1, tile_waves=2, xcd_remap=1)])
def test_forward_int32_64_images_4096(tdct, tune):
    """The int32 forward transform alone over the 64 images of 4096 x 4096
    (4 GiB of coefficients), in the launch shapes the autotuner picks for
    it; every image compared in full."""
    import torch
    sizes, seeds, qs = synth.large_batch_spec()
    n, side = len(sizes), sizes[0][0]
    buf, off, strides = synth.batch(sizes, seeds)
    src = torch.from_numpy(buf).cuda()
    nblk = (side // 8) ** 2
    Y = torch.empty((n, nblk, 64), dtype=torch.int32, device="cuda")
    base = src.data_ptr()
    descs = [tdct.image_desc(tdct.OP_FORWARD, side, side, src=base + int(off[i]), src_stride=side,
                             coef=Y[i]) for i in range(n)]
    plan = tdct.tdct_batch_plan(descs, qs, tune=tune)
    try:
        tdct.tdct_batch_run(plan)
        sync()
        yh = Y.cpu().numpy()

        def check(i):
            img = synth.batch_view(buf, off, strides, sizes, i)
            return bool(np.array_equal(yh[i], O.forward(img)))

        with ThreadPoolExecutor(HOST_THREADS) as ex:
            ok = list(ex.map(check, range(n)))
        assert all(ok), [i for i, g in enumerate(ok) if not g]
    finally:
        tdct.tdct_plan_free(plan)
        del Y
        torch.cuda.empty_cache()


def test_ragged_10000_images_one_persistent_launch(tdct):
    """10,000 images with log-uniform sides in [64, 2048]: full encode +
    decode round trip with coefficients, one launch from the block-offset
    table, replayed through a graph, against one plain launch per image and
    one launch with cached pixel accesses."""
    import torch
    sizes, seeds, qs = synth.ragged_batch_spec()
    n = len(sizes)
    buf, off, strides = synth.batch(sizes, seeds)
    src = torch.from_numpy(buf).cuda()
    nblk = np.array([(w // 8) * (h // 8) for w, h in sizes], np.int64)
    boff = np.concatenate([[0], np.cumsum(nblk)])
    coef = torch.empty((int(boff[-1]), 64), dtype=torch.int16, device="cuda")
    dst = torch.zeros(buf.size, dtype=torch.uint8, device="cuda")  # gaps between images stay 0
    base, cb, db = src.data_ptr(), coef.data_ptr(), dst.data_ptr()
    descs = [tdct.image_desc(tdct.OP_ROUNDTRIP, w, h, qtab=i, keep=64, src=base + int(off[i]),
                             src_stride=w, coef=cb + 128 * int(boff[i]), dst=db + int(off[i]),
                             dst_stride=w) for i, (w, h) in enumerate(sizes)]
    plan = tdct.tdct_batch_plan(descs, qs)
    try:
        tdct.tdct_batch_graph(plan)
        tdct.tdct_batch_graph(plan)
        sync()
        dh = dst.cpu().numpy()
        ch = coef.cpu().numpy()

        def check(i):  # every image in full
            img = synth.batch_view(buf, off, strides, sizes, i)
            q_ref, rec_ref = O.roundtrip(img, qs[i])
            return bool(np.array_equal(ch[boff[i]:boff[i + 1]], q_ref) and
                        np.array_equal(synth.batch_view(dh, off, strides, sizes, i), rec_ref))

        with ThreadPoolExecutor(HOST_THREADS) as ex:
            ok = list(ex.map(check, range(n)))
        assert all(ok), [i for i, g in enumerate(ok) if not g][:20]
        # one plain launch per image writes the very same bytes
        coef2 = torch.empty_like(coef)
        dst2 = torch.zeros_like(dst)
        d2 = [tdct.image_desc(tdct.OP_ROUNDTRIP, w, h, qtab=i, keep=64, src=base + int(off[i]),
                              src_stride=w, coef=coef2.data_ptr() + 128 * int(boff[i]),
                              dst=dst2.data_ptr() + int(off[i]), dst_stride=w)
              for i, (w, h) in enumerate(sizes)]
        tdct.tdct_run_per_image(d2, qs)
        sync()
        assert torch.equal(coef, coef2) and torch.equal(dst, dst2)
        # and so does the launch shape the autotuner picks for this batch (XCD
        # order, cached pixel accesses)
        coef2.zero_()
        dst2.zero_()
        tune = dict(waves_per_group=1, groups_per_cu=4096, tile_waves=1, xcd_remap=1, pixel_cache=1)
        p2 = tdct.tdct_batch_plan(d2, qs, tune=tune)
        try:
            tdct.tdct_batch_run(p2)
            sync()
        finally:
            tdct.tdct_plan_free(p2)
        assert torch.equal(coef, coef2) and torch.equal(dst, dst2)
    finally:
        tdct.tdct_plan_free(plan)


def test_video_420_frames_int8_zigzag(tdct):
    """All 256 frames of 3840 x 2160 4:2:0 in one batched launch with
    luma/chroma Q tables, every plane compared with the oracle."""
    import torch
    v = synth.Video420()
    frames = list(range(v.frames))
    planes, descs, qtabs, outs = [], [], [], []
    for k, f in enumerate(frames):
        Y, Cb, Cr = v.frame(f)
        qy, qc = v.qtables(f)
        qtabs += [qy, qc]
        for p, (pl, qi) in enumerate([(Y, 2 * k), (Cb, 2 * k + 1), (Cr, 2 * k + 1)]):
            h, w = pl.shape
            d = torch.from_numpy(pl).cuda()
            o = torch.empty(((w // 8) * (h // 8), 64), dtype=torch.int8, device="cuda")
            planes.append((pl, qi))
            outs.append(o)
            descs.append(tdct.image_desc(tdct.OP_ENCODE_I8ZZ, w, h, qtab=qi, src=d, src_stride=w, coef=o))
            outs.append(d)
    plan = tdct.tdct_batch_plan(descs, qtabs)
    try:
        tdct.tdct_batch_run(plan)
        sync()
        got = [outs[2 * j].cpu().numpy() for j in range(len(planes))]

        def check(j):
            pl, qi = planes[j]
            return bool(np.array_equal(got[j], O.quantise_i8_zigzag(pl, qtabs[qi])))

        with ThreadPoolExecutor(HOST_THREADS) as ex:
            ok = list(ex.map(check, range(len(planes))))
        assert all(ok), [j for j, g in enumerate(ok) if not g][:20]
    finally:
        tdct.tdct_plan_free(plan)
