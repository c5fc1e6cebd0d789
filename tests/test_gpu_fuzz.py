"""Seeded random cases through every plain entry point, against the oracle.

Each case draws an operation, a size (multiples of 8 up to 320 on a side,
so several wave-tiles and ragged tails), a row stride (aligned or not), a
byte offset of the plane from an aligned allocation, a quantisation table
(unit, random over [1, 4095], small, the paper-style 1 + s(i + j), or all
4095), a zonal keep, and an input (textured, uniform random bytes, extreme
0/255 patterns; for the decoder, int16 coefficients over the full range or
near zero). Outputs sit between guard bands that must stay untouched, and
every element must equal the oracle's (tolerance 0).
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_helpers import Guarded, plane_dev, sync, to_dev

pytestmark = pytest.mark.gpu

CASES = 120
OPS = ("quantise", "inverse", "roundtrip_q", "roundtrip", "forward", "i8zz")


@pytest.fixture(scope="module")
def tdct():
    import paper_1702_00817_amd as m
    return m


def _qtable(rng):
    kind = rng.integers(5)
    if kind == 0:
        return np.ones(64, np.uint16)
    if kind == 1:
        return rng.integers(1, 4096, size=64).astype(np.uint16)
    if kind == 2:
        return rng.integers(1, 17, size=64).astype(np.uint16)
    if kind == 3:
        return synth.qtable(1, int(rng.integers(1, 9)))
    return np.full(64, 4095, np.uint16)


def _plane(rng, w, h, stride):
    kind = rng.integers(3)
    if kind == 0:
        return synth.textured(w, h, int(rng.integers(1 << 30)), stride=stride)
    if kind == 1:
        return rng.integers(0, 256, size=(h, stride)).astype(np.uint8)
    return np.where(rng.random((h, stride)) < 0.5, 0, 255).astype(np.uint8)


def _coefs(rng, nblk):
    if rng.integers(2):
        return rng.integers(-32768, 32768, size=(nblk, 64)).astype(np.int16)
    return rng.integers(-40, 41, size=(nblk, 64)).astype(np.int16)


def _case(seed):
    rng = np.random.default_rng(seed)
    op = OPS[seed % len(OPS)]
    w = 8 * int(rng.integers(1, 41))
    h = 8 * int(rng.integers(1, 41))
    stride = w + (int(rng.integers(0, 18)) if rng.integers(2) else 8 * int(rng.integers(0, 4)))
    offset = int(rng.integers(0, 16)) if rng.integers(2) else 0
    return rng, op, w, h, stride, offset


@pytest.mark.parametrize("seed", range(CASES))
def test_random_case_matches_oracle(tdct, seed):
    rng, op, w, h, stride, offset = _case(seed)
    Q = _qtable(rng)
    keep = int(rng.integers(1, 65)) if rng.integers(2) else 64
    nblk = (w // 8) * (h // 8)
    print("case", seed, op, w, h, stride, offset, keep, flush=True)
    if op == "inverse":
        q = _coefs(rng, nblk)
        qd = to_dev(q)
        out = Guarded(h * stride, offset=offset)
        tdct.tdct_inverse(qd.data_ptr(), Q, w, h, out.ptr, stride)
        sync()
        assert out.guards_intact()
        rec = out.host().reshape(h, stride)
        assert np.array_equal(rec[:, :w], O.inverse(q, Q, w, h))
        assert (rec[:, w:] == out.fill).all(), "bytes between rows were written"
        return
    img = _plane(rng, w, h, stride)
    _, sp = plane_dev(img, offset)
    if op == "quantise":
        out = Guarded(nblk * 128)
        tdct.tdct_quantise(sp, stride, w, h, Q, keep, out.ptr)
        sync()
        assert out.guards_intact()
        assert np.array_equal(out.host().view(np.int16).reshape(nblk, 64), O.quantise(img, Q, keep, w=w))
    elif op in ("roundtrip_q", "roundtrip"):
        qo = Guarded(nblk * 128) if op == "roundtrip_q" else None
        out = Guarded(h * stride)
        tdct.tdct_roundtrip(sp, stride, w, h, Q, keep, qo.ptr if qo else None, out.ptr, stride)
        sync()
        q_ref, rec_ref = O.roundtrip(img, Q, keep, w=w)
        assert out.guards_intact()
        rec = out.host().reshape(h, stride)
        assert np.array_equal(rec[:, :w], rec_ref)
        assert (rec[:, w:] == out.fill).all(), "bytes between rows were written"
        if qo:
            assert qo.guards_intact()
            assert np.array_equal(qo.host().view(np.int16).reshape(nblk, 64), q_ref)
    elif op == "forward":
        out = Guarded(nblk * 256)
        tdct.tdct_forward(sp, stride, w, h, out.ptr)
        sync()
        assert out.guards_intact()
        assert np.array_equal(out.host().view(np.int32).reshape(nblk, 64), O.forward(img, w=w))
    else:
        out = Guarded(nblk * 64)
        tdct.tdct_quantise_i8_zigzag(sp, stride, w, h, Q, out.ptr)
        sync()
        assert out.guards_intact()
        assert np.array_equal(out.host().view(np.int8).reshape(nblk, 64), O.quantise_i8_zigzag(img, Q, w=w))


def test_cases_cover_every_op_and_layout():
    """The seeded draw exercises each entry point, unaligned strides and
    offsets, ragged tiles (more than 128 blocks, not a multiple of 128)."""
    seen = set()
    unaligned = ragged = 0
    for seed in range(CASES):
        _, op, w, h, stride, offset = _case(seed)
        seen.add(op)
        unaligned += (stride % 8 != 0) or (offset % 8 != 0)
        nblk = (w // 8) * (h // 8)
        ragged += nblk > 128 and nblk % 128 != 0
    assert seen == set(OPS)
    assert unaligned >= 20 and ragged >= 40
