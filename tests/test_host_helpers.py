"""The library's device building blocks, compiled for the host and checked
on the CPU: the operation count of Table 1, the 1-D and 2-D butterflies
against the oracle's dense products, the zigzag scan, the D^2 shift table,
and the float quantiser over its entire input domain."""
import ctypes
import itertools
import os

import numpy as np
import pytest

from conftest import ROOT

HC = os.path.join(ROOT, "tests", "libhostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(HC):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "tdct_build", os.path.join(ROOT, "paper_1702_00817_amd", "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build_hostcheck()
    L = ctypes.CDLL(HC)
    P = ctypes.c_void_p
    L.hc_count.argtypes = [ctypes.c_int32, ctypes.c_int32, P]
    L.hc_apply8.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32]
    L.hc_apply8x8.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32]
    L.hc_zigzag.argtypes = [P]
    L.hc_shifts.argtypes = [P]
    L.hc_quant.argtypes = [ctypes.c_int32] * 4 + [P]
    L.hc_quant_lanes.argtypes = [ctypes.c_int32] * 4 + [P, P]
    L.hc_xcd_order.argtypes = [ctypes.c_uint32, P]
    L.hc_inverse_f32.argtypes = [P, ctypes.c_int64, P, P]
    return L


def _counts(hc, inverse, block):
    c = np.zeros(5, np.int32)
    hc.hc_count(inverse, block, c.ctypes.data)
    return dict(zip(("add", "sub", "neg", "mul", "shift"), c.tolist()))


@pytest.mark.parametrize("inverse", [0, 1])
def test_one_pass_costs_14_additions_no_mult_no_shift(hc, inverse):
    c = _counts(hc, inverse, 0)
    assert c["add"] + c["sub"] == 14
    assert c["neg"] == 0 and c["mul"] == 0 and c["shift"] == 0


@pytest.mark.parametrize("inverse", [0, 1])
def test_block_transform_costs_16_passes(hc, inverse):
    c = _counts(hc, inverse, 1)
    assert c["add"] + c["sub"] == 16 * 14 and c["neg"] == c["mul"] == c["shift"] == 0


def _apply8(hc, X, inverse):
    X = np.ascontiguousarray(X, np.int64)
    out = np.zeros_like(X)
    hc.hc_apply8(X.ctypes.data, out.ctypes.data, X.shape[0], inverse)
    return out


def test_butterflies_equal_dense_T_on_all_3pow8_vectors(hc, oracle_mod):
    V = np.array(list(itertools.product((-1, 0, 1), repeat=8)), np.int64)
    T = oracle_mod.T().astype(np.int64)
    assert np.array_equal(_apply8(hc, V, 0), V @ T.T)
    assert np.array_equal(_apply8(hc, V, 1), V @ T)
    # and through the oracle's own 1-D routine on a sample
    for v in V[::97]:
        assert np.array_equal(_apply8(hc, v[None], 0)[0], oracle_mod.apply_T(v))
        assert np.array_equal(_apply8(hc, v[None], 1)[0], oracle_mod.apply_T(v, True))


def test_butterflies_equal_dense_T_on_random_int16(hc, oracle_mod):
    rng = np.random.default_rng(21)
    V = rng.integers(-32768, 32768, size=(1_000_000, 8))
    T = oracle_mod.T().astype(np.int64)
    assert np.array_equal(_apply8(hc, V, 0), V @ T.T)
    assert np.array_equal(_apply8(hc, V, 1), V @ T)


def test_2d_butterfly_equals_oracle_block_products(hc, oracle_mod):
    rng = np.random.default_rng(22)
    X = rng.integers(-128, 128, size=(300, 64))
    out = np.zeros_like(X)
    hc.hc_apply8x8(np.ascontiguousarray(X).ctypes.data, out.ctypes.data, X.shape[0], 0)
    W = rng.integers(-5000, 5000, size=(300, 64))
    outi = np.zeros_like(W)
    hc.hc_apply8x8(np.ascontiguousarray(W).ctypes.data, outi.ctypes.data, W.shape[0], 1)
    for k in range(X.shape[0]):
        assert np.array_equal(out[k].reshape(8, 8), oracle_mod.forward_block(X[k].reshape(8, 8)))
        assert np.array_equal(outi[k].reshape(8, 8), oracle_mod.inverse_block(W[k].reshape(8, 8)))


def test_zigzag_table_matches_oracle(hc, oracle_mod):
    z = np.zeros(64, np.int32)
    hc.hc_zigzag(z.ctypes.data)
    assert np.array_equal(z, oracle_mod.zigzag_order())


def test_shift_table_is_log2_of_oracle_scale(hc, oracle_mod):
    s = np.zeros(64, np.int32)
    hc.hc_shifts(s.ctypes.data)
    assert np.array_equal(1 << s, oracle_mod.wscale().reshape(-1))
    assert s.min() == 0 and s.max() == 4


def test_float_quantiser_is_exact_on_the_whole_encoder_domain(hc, oracle_mod):
    """Every (y, s, Q) the encoder can meet: |y * 2^s| <= 8192, s in 0..4,
    Q in 1..4095, against the oracle's exact rational rounding."""
    bad = []
    for s in range(5):
        lim = 8192 >> s
        y = np.arange(-lim, lim + 1, dtype=np.int64)
        W = y << s
        out = np.zeros(y.size, np.int32)
        for Q in range(1, 4096):
            hc.hc_quant(Q, s, -lim, y.size, out.ctypes.data)
            exp = oracle_mod.round_div_array(W, Q)
            if not np.array_equal(out, exp):
                k = int(np.nonzero(out != exp)[0][0])
                bad.append((s, Q, int(W[k]), int(out[k]), int(exp[k])))
                break
    assert not bad, bad[:5]


def test_quantiser_lane_forms_store_the_right_bits(hc, oracle_mod):
    """The stored int16 halfword and the saturated int8 byte, taken straight
    from the float's bits, equal the rounded quotient (clamped for int8)."""
    rng = np.random.default_rng(31)
    for Q in [1, 2, 3, 63, 64, 65, 113, 4095] + rng.integers(1, 4096, 40).tolist():
        for s in range(5):
            lim = 8192 >> s
            y = np.arange(-lim, lim + 1, dtype=np.int64)
            o8 = np.zeros(y.size, np.int8)
            o16 = np.zeros(y.size, np.int16)
            hc.hc_quant_lanes(int(Q), s, -lim, y.size, o8.ctypes.data, o16.ctypes.data)
            exp = oracle_mod.round_div_array(y << s, int(Q))
            assert np.array_equal(o16.astype(np.int64), exp)
            assert np.array_equal(o8.astype(np.int64), np.clip(exp, -128, 127))


@pytest.mark.parametrize("n", list(range(1, 40)) + [255, 256, 257, 1023, 131072, 131075, 402064])
def test_xcd_order_is_a_bijection_with_one_contiguous_range_per_xcd(hc, n):
    """The batch kernel's XCD remap: workgroup b runs on XCD b % 8; its place
    in the tile order must be a permutation of [0, n) under which the
    workgroups of each XCD, in launch order, take one contiguous range, the
    ranges following XCD order."""
    out = np.zeros(n, np.uint32)
    hc.hc_xcd_order(n, out.ctypes.data)
    assert np.array_equal(np.sort(out), np.arange(n, dtype=np.uint32))
    nxt = 0
    for x in range(8):
        places = out[x::8]  # XCD x's workgroups in launch order
        assert np.array_equal(places, np.arange(nxt, nxt + places.size, dtype=np.uint32))
        nxt += places.size


def test_fp32_round_trip_decoder_is_exact(hc, oracle_mod):
    """The round trips decode in fp32. With q from the encoder |q Q| < 10240;
    over that whole range (random blocks, plus for every output the block
    whose signs drive that output to its extreme) the fp32 inverse of
    q Q / 64 with the pixel bias equals S / 64 + 128 + 1/128 exactly (S from
    the oracle's integer inverse), and rounding it to nearest with
    saturation gives the integer decoder's clamp(floor((S + 32) / 64) + 128)."""
    T = oracle_mod.T().astype(np.int64)
    rng = np.random.default_rng(61)
    blocks = [rng.integers(-10240, 10241, size=(4000, 64)),
              rng.integers(-300, 301, size=(4000, 64)),        # near the clamps
              np.full((1, 64), 10240), np.full((1, 64), -10240)]
    ext = []
    for r in range(8):
        for c in range(8):
            sg = np.sign(np.outer(T[:, r], T[:, c]))           # sign of T_ir T_jc
            ext += [10240 * sg, -10240 * sg]
    blocks.append(np.array(ext).reshape(-1, 64))
    wq = np.ascontiguousarray(np.concatenate(blocks).astype(np.int32))
    n = wq.shape[0]
    out = np.zeros((n, 64), np.float32)
    pix = np.zeros((n, 64), np.uint8)
    hc.hc_inverse_f32(wq.ctypes.data, n, out.ctypes.data, pix.ctypes.data)
    S = np.stack([oracle_mod.inverse_block(wq[b].reshape(8, 8)).reshape(64) for b in range(n)])
    # the extreme blocks reach the largest |S| there is: 10240 times the
    # number of nonzero T_ir T_jc, maximised over the output (r, c)
    nz = (T != 0).sum(axis=0)
    assert np.abs(S).max() == 10240 * int(nz.max()) ** 2
    np.testing.assert_array_equal(out.astype(np.float64), S / 64.0 + 128.0 + 1.0 / 128.0)
    want = np.clip(np.floor_divide(S + 32, 64) + 128, 0, 255)
    np.testing.assert_array_equal(pix, want)
