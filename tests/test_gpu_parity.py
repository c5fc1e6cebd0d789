"""HIP path vs the CPU oracle, element by element, through the C ABI.

Every comparison is exact (tolerance 0): the codec is integer arithmetic and
has exactly one correct output per input. Sizes span several wave-tiles and
ragged tails; edge cases cover strips, odd block counts per row, strides,
unaligned planes, saturating patterns and both ends of the Q range. Output
buffers carry sentinel guard bands that must stay untouched.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import Guarded, plane_dev, sync, to_dev

pytestmark = pytest.mark.gpu

T = None


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


def _rand_q(rng, lo=1, hi=4095):
    return rng.integers(lo, hi + 1, size=64).astype(np.uint16)


def _encode(tdct, img, Q, keep=64, w=None, offset=0):
    h = img.shape[0]
    w = img.shape[1] if w is None else w
    stride = img.shape[1]
    _, sp = plane_dev(img, offset)
    nblk = (w // 8) * (h // 8)
    out = Guarded(nblk * 128)
    tdct.tdct_quantise(sp, stride, w, h, Q, keep, out.ptr)
    sync()
    assert out.guards_intact()
    return out.host().view(np.int16).reshape(nblk, 64)


def _decode(tdct, q, Q, w, h, dst_stride=None, offset=0):
    dst_stride = w if dst_stride is None else dst_stride
    qd = to_dev(np.ascontiguousarray(q.astype(np.int16)))
    out = Guarded(h * dst_stride, offset=offset)
    tdct.tdct_inverse(qd.data_ptr(), Q, w, h, out.ptr, dst_stride)
    sync()
    assert out.guards_intact()
    rec = out.host().reshape(h, dst_stride)
    if dst_stride > w:
        assert (rec[:, w:] == out.fill).all(), "bytes between rows were written"
    return rec[:, :w]


SIZES = [(8, 8), (16, 8), (24, 16), (40, 24), (136, 72), (1024, 64), (520, 48), (8, 520),
         (2048, 16), (512, 512)]


@pytest.mark.parametrize("w,h", SIZES)
def test_encode_matches_oracle(tdct, w, h):
    rng = np.random.default_rng(w * 131 + h)
    img = synth.textured(w, h, 100 + w + h)
    for Q, keep in [(synth.qtable(1, 3), 64), (_rand_q(rng), 64), (np.ones(64, np.uint16), 10),
                    (_rand_q(rng, 1, 40), 1), (_rand_q(rng, 1, 9), 37)]:
        got = _encode(tdct, img, Q, keep)
        assert np.array_equal(got, O.quantise(img, Q, keep)), (w, h, keep)


@pytest.mark.parametrize("w,h", SIZES)
def test_decode_matches_oracle_on_arbitrary_int16(tdct, w, h):
    rng = np.random.default_rng(w * 7 + h)
    nblk = (w // 8) * (h // 8)
    for Q, q in [(_rand_q(rng), rng.integers(-32768, 32768, size=(nblk, 64))),
                 (synth.qtable(1, 5), rng.integers(-300, 301, size=(nblk, 64))),
                 (np.full(64, 4095, np.uint16),
                  np.where(rng.random((nblk, 64)) < 0.5, 32767, -32768))]:
        q = q.astype(np.int16)
        got = _decode(tdct, q, Q, w, h)
        assert np.array_equal(got, O.inverse(q, Q, w, h)), (w, h)


@pytest.mark.parametrize("w,h", [(8, 8), (136, 72), (512, 512), (24, 40)])
def test_encoder_output_decodes_like_oracle(tdct, w, h):
    img = synth.textured(w, h, 7 + w)
    Q = synth.qtable(1, 4)
    q = _encode(tdct, img, Q)
    rec = _decode(tdct, q, Q, w, h)
    q_ref, rec_ref = O.roundtrip(img, Q)
    assert np.array_equal(q, q_ref) and np.array_equal(rec, rec_ref)


def test_unit_Q_round_trip_is_identity_on_gpu(tdct):
    img = synth.textured(256, 64, 77)
    one = np.ones(64, np.uint16)
    rec = _decode(tdct, _encode(tdct, img, one), one, 256, 64)
    assert np.array_equal(rec, img)


@pytest.mark.parametrize("stride,offset", [(64, 0), (72, 0), (80, 0), (67, 0), (64, 3), (96, 8)])
def test_strides_and_alignment(tdct, stride, offset):
    w, h = 48, 24
    img = synth.textured(w, h, 31, stride=stride)
    Q = synth.qtable(1, 2)
    got = _encode(tdct, img, Q, w=w, offset=offset)
    ref = O.quantise(img, Q, 64, w=w)
    assert np.array_equal(got, ref)
    rec = _decode(tdct, ref, Q, w, h, dst_stride=stride, offset=offset)
    assert np.array_equal(rec, O.inverse(ref, Q, w, h))


def test_roundtrip_kernel(tdct):
    for (w, h), keep, with_q in [((136, 72), 64, True), ((512, 64), 10, False), ((24, 16), 25, True),
                                 ((8, 8), 1, True)]:
        img = synth.textured(w, h, 5 + w)
        Q = synth.qtable(1, 6)
        _, sp = plane_dev(img)
        nblk = (w // 8) * (h // 8)
        qo = Guarded(nblk * 128) if with_q else None
        out = Guarded(w * h)
        tdct.tdct_roundtrip(sp, w, w, h, Q, keep, qo.ptr if qo else None, out.ptr, w)
        sync()
        q_ref, rec_ref = O.roundtrip(img, Q, keep)
        assert out.guards_intact() and np.array_equal(out.host().reshape(h, w), rec_ref)
        if qo:
            assert qo.guards_intact()
            assert np.array_equal(qo.host().view(np.int16).reshape(nblk, 64), q_ref)


@pytest.mark.parametrize("w,h", [(2048, 2048), (2056, 2048)])
def test_plain_calls_on_both_sides_of_the_pixel_policy_size(tdct, w, h):
    """Plain calls take cached pixel accesses up to 4 Mpx and streaming ones
    above: 2048 x 2048 is exactly 4 Mpx, 2056 x 2048 just above. Encode, decode
    and the fused round trip (with coefficients) on a plane whose row stride is
    not a multiple of 128 bytes, every output against the oracle."""
    stride = w + 48
    img = synth.textured(w, h, w + h, stride=stride)
    Q = synth.qtable(1, 4)
    got = _encode(tdct, img, Q, w=w)
    ref = O.quantise(img, Q, 64, w=w)
    assert np.array_equal(got, ref)
    rec = _decode(tdct, ref, Q, w, h, dst_stride=stride)
    assert np.array_equal(rec, O.inverse(ref, Q, w, h))
    _, sp = plane_dev(img)
    nblk = (w // 8) * (h // 8)
    qo, out = Guarded(nblk * 128), Guarded(h * stride)
    tdct.tdct_roundtrip(sp, stride, w, h, Q, 10, qo.ptr, out.ptr, stride)
    sync()
    q_rt, rec_rt = O.roundtrip(img, Q, 10, w=w)
    assert qo.guards_intact() and out.guards_intact()
    assert np.array_equal(qo.host().view(np.int16).reshape(nblk, 64), q_rt)
    assert np.array_equal(out.host().reshape(h, stride)[:, :w], rec_rt)


def test_roundtrip_in_place(tdct):
    w, h = 64, 32
    img = synth.textured(w, h, 8)
    Q = synth.qtable(1, 1)
    d, p = plane_dev(img)
    tdct.tdct_roundtrip(p, w, w, h, Q, 64, None, p, w)
    sync()
    assert np.array_equal(d.cpu().numpy()[:w * h].reshape(h, w), O.roundtrip(img, Q)[1])


def test_forward_int32_and_psnr_single_image(tdct):
    """The 512 x 512 paper-sized case: int32 coefficients, zonal keep 10 with
    Q = 1, reconstruction and PSNR."""
    import torch
    img = synth.single_image()
    _, sp = plane_dev(img)
    Y = Guarded(4096 * 256)
    tdct.tdct_forward(sp, 512, 512, 512, Y.ptr)
    one = np.ones(64, np.uint16)
    rec = Guarded(512 * 512)
    tdct.tdct_roundtrip(sp, 512, 512, 512, one, 10, None, rec.ptr, 512)
    sse = torch.zeros(1, dtype=torch.int64, device="cuda")
    tdct.tdct_sse(sp, 512, rec.ptr, 512, 512, 512, sse.data_ptr())
    sync()
    assert Y.guards_intact() and rec.guards_intact()
    assert np.array_equal(Y.host().view(np.int32).reshape(4096, 64), O.forward(img))
    rec_ref = O.roundtrip(img, one, 10)[1]
    assert np.array_equal(rec.host().reshape(512, 512), rec_ref)
    assert int(sse.item()) == O.sse(img, rec_ref)
    assert O.psnr(img, rec_ref) == pytest.approx(10 * np.log10(255 ** 2 / (int(sse.item()) / img.size)))


@pytest.mark.parametrize("w,h", [(3840, 16), (1920, 8), (24, 24), (8, 8)])
def test_i8_zigzag_encoder(tdct, w, h):
    img = synth.textured(w, h, 44 + w)
    for Q in (synth.qtable(64, 3), synth.qtable(64, 5, step=2), synth.qtable(1, 1)):
        _, sp = plane_dev(img)
        nblk = (w // 8) * (h // 8)
        out = Guarded(nblk * 64)
        tdct.tdct_quantise_i8_zigzag(sp, w, w, h, Q, out.ptr)
        sync()
        assert out.guards_intact()
        assert np.array_equal(out.host().view(np.int8).reshape(nblk, 64), O.quantise_i8_zigzag(img, Q))


def test_constant_planes_and_saturating_patterns(tdct, oracle_mod):
    T = oracle_mod.T()
    tiles = []
    for i in range(8):
        for j in range(8):
            sgn = np.outer(T[i], T[j])
            for s in (1, -1):
                tiles.append(np.where(sgn * s > 0, 255, np.where(sgn * s < 0, 0, 128)).astype(np.uint8))
    img = np.concatenate([np.concatenate(tiles[k:k + 16], axis=1) for k in range(0, 128, 16)], axis=0)
    cases = [img, np.zeros((64, 64), np.uint8), np.full((64, 64), 255, np.uint8)]
    for im in cases:
        h, w = im.shape
        for Q in (np.ones(64, np.uint16), np.full(64, 4095, np.uint16), synth.qtable(1, 8)):
            q = _encode(tdct, im, Q)
            assert np.array_equal(q, O.quantise(im, Q))
            assert np.array_equal(_decode(tdct, q, Q, w, h), O.inverse(q, Q, w, h))
            # the round trips decode in fp32 and saturate in the u8 conversion:
            # these patterns overshoot both ends of [0, 255]
            _, sp = plane_dev(im)
            for keep in (64, 3):
                q_ref, rec_ref = O.roundtrip(im, Q, keep)
                for with_q in (True, False):
                    qo = Guarded(w * h * 2) if with_q else None
                    out = Guarded(w * h)
                    tdct.tdct_roundtrip(sp, w, w, h, Q, keep, qo.ptr if qo else None, out.ptr, w)
                    sync()
                    assert out.guards_intact() and np.array_equal(out.host().reshape(h, w), rec_ref)
                    if qo:
                        assert qo.guards_intact()
                        assert np.array_equal(qo.host().view(np.int16).reshape(-1, 64), q_ref)
    Y = O.forward(img).astype(np.int64)
    W = Y * oracle_mod.wscale().reshape(1, 64)
    assert Y[:, 0].min() == -8192 and Y[:, 0].max() == 8128  # the DC extremes are reached
    assert np.abs(W).max() == 8192  # and so is the bound on every scaled coefficient


def test_error_codes(tdct):
    import torch
    buf = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    p = buf.data_ptr()
    Q = synth.qtable(1, 1)
    lib = tdct.lib()
    q = tdct.qtable(Q)
    import ctypes
    r = ctypes.byref
    assert lib.tdct_quantise(None, 8, 8, 8, r(q), 64, p, None) == tdct.TDCT_EINVAL
    assert lib.tdct_quantise(p, 8, 12, 8, r(q), 64, p, None) == tdct.TDCT_EDIM
    assert lib.tdct_quantise(p, 8, 8, 0, r(q), 64, p, None) == tdct.TDCT_EDIM
    assert lib.tdct_quantise(p, 4, 8, 8, r(q), 64, p, None) == tdct.TDCT_EINVAL
    assert lib.tdct_quantise(p, 8, 8, 8, r(q), 0, p, None) == tdct.TDCT_EINVAL
    assert lib.tdct_quantise(p, 8, 8, 8, r(q), 65, p, None) == tdct.TDCT_EINVAL
    assert lib.tdct_quantise(p, 8, 8, 8, r(q), 64, p + 2, None) == tdct.TDCT_EINVAL
    bad = tdct.qtable(Q)
    bad.q[5] = 0
    assert lib.tdct_quantise(p, 8, 8, 8, r(bad), 64, p, None) == tdct.TDCT_EQTAB
    bad.q[5] = 4096
    assert lib.tdct_inverse(p, r(bad), 8, 8, p, 8, None) == tdct.TDCT_EQTAB
    assert lib.tdct_inverse(p, r(q), 8, 8, None, 8, None) == tdct.TDCT_EINVAL
    with pytest.raises(tdct.TdctError):
        tdct.tdct_quantise(p, 8, 9, 8, Q, 64, p)
    sync()


def test_stream_probes_move_the_bytes(tdct):
    import torch
    units = 4096 + 17
    a = torch.randint(0, 256, (2 * units * 16,), dtype=torch.uint8, device="cuda")
    b = torch.zeros_like(a)
    tdct.tdct_stream_probe(tdct.PROBE_COPY, a, b, units)
    sync()
    assert torch.equal(b[:units * 16], a[:units * 16]) and (b[units * 16:] == 0).all()
    tdct.tdct_stream_probe(tdct.PROBE_R1W2, a, b, units)
    sync()
    av = a[:units * 16]
    assert torch.equal(b[:units * 16], av) and torch.equal(b[units * 16:], av)
    tdct.tdct_stream_probe(tdct.PROBE_R2W1, a, b, units)
    sync()
    assert torch.equal(b[:units * 16], a[:units * 16] ^ a[units * 16:])
    with pytest.raises(tdct.TdctError):
        tdct.tdct_stream_probe(9, a, b, units)


def _sampled_blocks_match(img_dev, w, h, q_dev, rec_dev, Q, nsample, seed):
    """Checks sampled blocks (plus the four corners) of a large encode/decode
    against the oracle, each recomputed from its own 8x8 pixels."""
    rng = np.random.default_rng(seed)
    nbx, nby = w // 8, h // 8
    picks = [(0, 0), (nbx - 1, 0), (0, nby - 1), (nbx - 1, nby - 1)]
    picks += list(zip(rng.integers(0, nbx, nsample).tolist(), rng.integers(0, nby, nsample).tolist()))
    Q = np.asarray(Q)
    for bx, by in picks:
        blk = img_dev[8 * by:8 * by + 8, 8 * bx:8 * bx + 8].cpu().numpy()
        q_ref, rec_ref = O.roundtrip(np.ascontiguousarray(blk), Q)
        b = by * nbx + bx
        assert np.array_equal(q_dev[b].cpu().numpy(), q_ref[0]), (bx, by)
        assert np.array_equal(rec_dev[8 * by:8 * by + 8, 8 * bx:8 * bx + 8].cpu().numpy(), rec_ref), (bx, by)


@pytest.mark.parametrize("w,h", [(65536, 64), (64, 65536), (8, 8192), (8192, 8), (65536, 65536)])
def test_maximum_sides(tdct, w, h):
    """Sides up to the 65536 limit; the last case holds 2^32 pixels, so byte
    offsets of pixels and coefficients pass 2^32."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(w * 7 + h)
    img = torch.randint(0, 256, (h, w), dtype=torch.uint8, device="cuda", generator=g)
    nblk = (w // 8) * (h // 8)
    q = torch.empty((nblk, 64), dtype=torch.int16, device="cuda")
    rec = torch.empty((h, w), dtype=torch.uint8, device="cuda")
    Q = synth.qtable(1, 2)
    tdct.tdct_quantise(img, w, w, h, Q, 64, q)
    tdct.tdct_inverse(q, Q, w, h, rec, w)
    sync()
    _sampled_blocks_match(img, w, h, q, rec, Q, 300, w + h)
    del q, rec
    torch.cuda.empty_cache()
    # the int32 forward transform over the same plane (up to 16 GiB of output)
    Y = torch.empty((nblk, 64), dtype=torch.int32, device="cuda")
    tdct.tdct_forward(img, w, w, h, Y)
    sync()
    nbx, nby = w // 8, h // 8
    rng = np.random.default_rng(w + 3 * h)
    picks = [(0, 0), (nbx - 1, nby - 1), (nbx - 1, 0), (0, nby - 1)]
    picks += list(zip(rng.integers(0, nbx, 300).tolist(), rng.integers(0, nby, 300).tolist()))
    for bx, by in picks:
        blk = np.ascontiguousarray(img[8 * by:8 * by + 8, 8 * bx:8 * bx + 8].cpu().numpy())
        assert np.array_equal(Y[by * nbx + bx].cpu().numpy(), O.forward(blk)[0]), (bx, by)
    del img, Y
    torch.cuda.empty_cache()
