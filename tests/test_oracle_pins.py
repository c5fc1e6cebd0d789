"""Pins for the CPU oracle: facts fixed by the paper and by mathematics,
none of them a re-typing of the oracle's own formulas.

T and its scaling (Section 2), the factorisation and its cost (Section 2,
Table 1), the block transform, zonal coding and reconstruction (Section 3)
are each checked against something other than the oracle: printed factor
matrices, orthogonality, closed forms, Parseval, brute force over small
domains and the paper's real-valued formulation.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

from conftest import GOLDEN, read_matrices, read_table

import synth

pytestmark = pytest.mark.filterwarnings("ignore")

FACTORS = read_matrices("paper_factors.txt")


def _factor_T(f=FACTORS):
    return f["P"] @ f["A3"] @ f["A2"] @ f["A1"]


# ---- Section 2: T, D, factorisation ---------------------------------------

def pin_printed_factors_multiply_to_oracle_T(O):
    assert np.array_equal(_factor_T(), O.T())


def pin_T_rows_orthogonal_with_norms_8_2_4_2(O):
    T = O.T().astype(np.int64)
    assert np.array_equal(T @ T.T, np.diag([8, 2, 4, 2, 8, 2, 4, 2]))


def pin_scaled_transform_orthogonal_with_printed_D(O):
    inv_d2 = np.array(read_table("paper_scaling.txt")[0], float)
    D = np.diag(1.0 / np.sqrt(inv_d2))
    C = D @ O.T()
    assert np.allclose(C @ C.T, np.eye(8), atol=1e-12)
    assert np.allclose(D, O.paper_D(), atol=0)


def pin_D2_is_powers_of_two_and_folds_to_integer_scale(O):
    inv_d2 = np.array(read_table("paper_scaling.txt")[0], np.int64)
    assert set((Fraction(1, int(v)) for v in inv_d2)) <= {Fraction(1, 2), Fraction(1, 4), Fraction(1, 8)}
    expect = np.array([[Fraction(64, int(a * b)) for b in inv_d2] for a in inv_d2])
    assert all(x.denominator == 1 for x in expect.ravel())
    assert np.array_equal(O.wscale(), expect.astype(np.int64))


def test_factorisation_costs_14_additions_like_table_1():
    rows = {r[0]: [int(v) for v in r[1:]] for r in read_table("table1_complexity.txt")
            if r[0] in ("proposed",)}
    adds = 0
    mults = 0
    for name in ("A1", "A2", "A3"):
        A = FACTORS[name]
        nz = (A != 0).sum(axis=1)
        adds += int((nz - 1).sum())
        mults += int(((np.abs(A) != 1) & (A != 0)).sum())
    # P only relabels: one 1 per row and column.
    P = FACTORS["P"]
    assert (P.sum(0) == 1).all() and (P.sum(1) == 1).all()
    assert [adds, mults, 0, adds + mults] == rows["proposed"]


def test_cost_percentages_in_text_follow_from_table_1():
    tab = read_table("table1_complexity.txt")
    total = {r[0]: int(r[4]) for r in tab if len(r) == 5}
    for kind, vs, pct in (r for r in tab if len(r) == 3):
        p = float(pct)
        val = (1 - total["proposed"] / total[vs]) if kind == "lower" else total["proposed"] / total[vs]
        assert abs(100 * val - p) < 0.05, (kind, vs)


def _apply_factors(f, x, transpose=False):
    x = np.asarray(x, np.int64)
    if not transpose:
        for name in ("A1", "A2", "A3", "P"):
            x = f[name] @ x
    else:
        for name in ("P", "A3", "A2", "A1"):
            x = f[name].T @ x
    return x


def pin_sparse_factor_path_equals_dense_on_all_3pow8_vectors(O):
    for v in itertools.product((-1, 0, 1), repeat=8):
        assert np.array_equal(_apply_factors(FACTORS, v), O.apply_T(v))
        assert np.array_equal(_apply_factors(FACTORS, v, True), O.apply_T(v, True))


def pin_sparse_factor_path_equals_dense_on_random_int16(O):
    rng = np.random.default_rng(11)
    for _ in range(3000):
        v = rng.integers(-32768, 32768, size=8)
        assert np.array_equal(_apply_factors(FACTORS, v), O.apply_T(v))
        assert np.array_equal(_apply_factors(FACTORS, v, True), O.apply_T(v, True))


# ---- Section 3: 2-D block transform ---------------------------------------

def pin_impulse_block_gives_outer_product_of_T_columns(O):
    """Y = T X T^t with X = e_r e_c^t is (column r of T)(column c of T)^t: fixes
    which side T multiplies and that it is not transposed."""
    T = _factor_T()
    for r in range(8):
        for c in range(8):
            X = np.zeros((8, 8), np.int64)
            X[r, c] = 1
            assert np.array_equal(O.forward_block(X), np.outer(T[:, r], T[:, c]))


def pin_horizontal_pattern_only_in_first_coefficient_row(O):
    """A block whose rows are all equal varies horizontally only, so only
    i = 0 (vertical DC) is non-zero and Y[0, j] = 8 (T f)_j."""
    T = _factor_T()
    rng = np.random.default_rng(3)
    for _ in range(20):
        f = rng.integers(-128, 128, size=8)
        X = np.tile(f, (8, 1))
        Y = O.forward_block(X)
        assert (Y[1:] == 0).all()
        assert np.array_equal(Y[0], 8 * (T @ f))


def pin_dc_is_level_shifted_block_sum(O):
    img = synth.textured(64, 48, 5)
    Y = O.forward(img)
    blocks = img.reshape(6, 8, 8, 8).transpose(0, 2, 1, 3).reshape(-1, 64).astype(np.int64)
    assert np.array_equal(Y[:, 0], (blocks - 128).sum(1))


def pin_constant_offset_changes_only_dc(O):
    rng = np.random.default_rng(4)
    img = rng.integers(0, 200, size=(32, 40), dtype=np.uint8)
    Y0 = O.forward(img).astype(np.int64)
    Y1 = O.forward((img + 37).astype(np.uint8)).astype(np.int64)
    d = Y1 - Y0
    assert (d[:, 0] == 64 * 37).all() and (d[:, 1:] == 0).all()


def pin_integer_parseval(O):
    """C = D Y D is orthonormal (Section 2), so sum C^2 = sum X^2, i.e.
    sum_ij W_ij Y_ij = 64 sum X^2 with W = 64 d_i^2 d_j^2 Y."""
    rng = np.random.default_rng(5)
    ws = O.wscale().astype(np.int64)
    for _ in range(200):
        X = rng.integers(-128, 128, size=(8, 8))
        Y = O.forward_block(X)
        assert int((ws * Y * Y).sum()) == 64 * int((X * X).sum())


def pin_scaled_coefficients_stay_within_8192(O):
    """|W| <= 64 * 128 for pixels in [0, 255]; the DC reaches -8192 and 8128."""
    T = O.T().astype(np.int64)
    ws = O.wscale().astype(np.int64)
    worst = 0
    for i in range(8):
        for j in range(8):
            sgn = np.outer(T[i], T[j])
            for s in (1, -1):
                X = np.where(sgn * s > 0, 127, np.where(sgn * s < 0, -128, 0))
                W = ws * O.forward_block(X)
                worst = max(worst, int(np.abs(W).max()))
    assert worst <= 8192
    lo = O.forward(np.zeros((8, 8), np.uint8))[0, 0]
    hi = O.forward(np.full((8, 8), 255, np.uint8))[0, 0]
    assert (lo, hi) == (-8192, 8128)


# ---- zonal coding (Section 3) ---------------------------------------------

def pin_zigzag_is_the_jpeg_scan(O):
    order = O.zigzag_order()
    assert sorted(order.tolist()) == list(range(64))
    ij = [(k // 8, k % 8) for k in order]
    assert ij[:6] == [(0, 0), (0, 1), (1, 0), (2, 0), (1, 1), (0, 2)]
    diag = [i + j for i, j in ij]
    assert diag == sorted(diag)
    for d in range(15):
        rows = [i for (i, j) in ij if i + j == d]
        assert rows == (sorted(rows) if d % 2 else sorted(rows, reverse=True))
    assert {k for k in order[:10]} == {8 * i + j for i in range(8) for j in range(8) if i + j <= 3}
    assert ij[-1] == (7, 7)


def test_compression_ratios_match_section_3():
    for r, pct in read_table("compression_ratios.txt"):
        assert abs(100 * (64 - int(r)) / 64 - float(pct)) < 0.005  # printed to ~2 decimals


def pin_zonal_keep_zeroes_exactly_the_tail(O):
    img = synth.textured(64, 64, 9)
    Q = np.ones(64)
    rank = O.zigzag_rank()
    full = O.quantise(img, Q, 64)
    for keep in (1, 2, 10, 25, 45, 63):
        q = O.quantise(img, Q, keep)
        assert (q[:, rank >= keep] == 0).all()
        assert np.array_equal(q[:, rank < keep], full[:, rank < keep])


# ---- quantiser ---------------------------------------------------------------

def _half_away(W, Q):
    f = Fraction(abs(W), Q) + Fraction(1, 2)
    m = f.numerator // f.denominator
    return -m if W < 0 else m


def pin_round_div_matches_rational_rounding(O):
    rng = np.random.default_rng(6)
    cases = [(W, Q) for Q in (1, 2, 3, 4, 7, 64, 113, 4095) for W in range(-300, 301)]
    cases += [(int(W), int(Q)) for W, Q in zip(rng.integers(-8192, 8193, 3000), rng.integers(1, 4096, 3000))]
    for W, Q in cases:
        assert O.round_div(W, Q) == _half_away(W, Q), (W, Q)


def pin_round_div_ties_go_away_from_zero_and_is_idempotent(O):
    for Q in (2, 4, 6, 100, 4094):
        assert O.round_div(Q // 2, Q) == 1
        assert O.round_div(-(Q // 2), Q) == -1
        assert O.round_div(Q // 2 - 1, Q) == 0
        for q in (-50, -3, 0, 1, 7, 99):
            assert O.round_div(q * Q, Q) == q


# ---- reconstruction ---------------------------------------------------------

def pin_unit_Q_full_keep_round_trip_is_exact(O):
    for seed, (w, h) in enumerate([(8, 8), (64, 40), (512, 64)]):
        img = synth.textured(w, h, 20 + seed)
        _, rec = O.roundtrip(img, np.ones(64), 64)
        assert np.array_equal(rec, img)
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, size=(40, 48), dtype=np.uint8)
    _, rec = O.roundtrip(img, np.ones(64), 64)
    assert np.array_equal(rec, img)


def pin_dc_only_block_closed_form(O):
    """With only W'_00 = v, S = v everywhere (row 0 of T is all ones), so every
    pixel is clamp(floor((v + 32) / 64) + 128); sweeps ties and both clamps."""
    vs = np.arange(-9000, 9001)
    q = np.zeros((vs.size, 64), np.int16)
    q[:, 0] = vs
    # lay the blocks out as one 8-pixel-high strip
    rec = O.inverse(q, np.ones(64), 8 * vs.size, 8)
    got = rec.reshape(8, vs.size, 8).transpose(1, 0, 2).reshape(vs.size, 64)
    expect = np.clip(np.floor_divide(vs + 32, 64) + 128, 0, 255)
    assert (got == expect[:, None]).all()


def pin_single_coefficient_block_closed_form(O):
    T = _factor_T()
    for i in range(8):
        for j in range(8):
            for v in (-640, -96, 32, 1000):
                q = np.zeros((1, 64), np.int16)
                q[0, 8 * i + j] = v
                rec = O.inverse(q, np.ones(64), 8, 8).astype(np.int64)
                S = v * np.outer(T[i], T[j])
                assert np.array_equal(rec, np.clip(np.floor_divide(S + 32, 64) + 128, 0, 255))


def pin_dequantise_multiplies_by_Q(O):
    rng = np.random.default_rng(12)
    q = rng.integers(-40, 41, size=(6, 64)).astype(np.int16)
    Q = rng.integers(1, 60, size=64).astype(np.uint16)
    a = O.inverse(q, Q, 48, 8)
    b = O.inverse((q.astype(np.int64) * Q).astype(np.int16), np.ones(64), 48, 8)
    assert np.array_equal(a, b)


def pin_integer_path_matches_paper_float_formulation(O):
    """With Q = 1 the integer reconstruction S / 64 equals the paper's
    C^t (mask o (C^ X C^t)) C^ (Section 3) with C^ = D T built from the
    printed D, for every zonal r."""
    rng = np.random.default_rng(13)
    ws = O.wscale().astype(np.int64)
    rank = O.zigzag_rank().reshape(8, 8)
    for _ in range(60):
        X = rng.integers(-128, 128, size=(8, 8))
        Y = O.forward_block(X)
        for r in (1, 2, 6, 10, 25, 35, 45, 64):
            Wm = np.where(rank < r, ws * Y, 0)
            S = O.inverse_block(Wm)
            ref = O.float_block_roundtrip(X, r)
            assert np.allclose(S / 64.0, ref, atol=1e-9)


def pin_plane_reconstruction_rounds_paper_float_result(O):
    img = synth.textured(32, 32, 14)
    for r in (2, 10, 25):
        _, rec = O.roundtrip(img, np.ones(64), r)
        for b in range(16):
            by, bx = divmod(b, 4)
            X = img[8 * by:8 * by + 8, 8 * bx:8 * bx + 8].astype(np.int64) - 128
            ref = O.float_block_roundtrip(X, r)
            # away from exact .5 ties the integer rule equals rounding the float
            frac = ref - np.floor(ref)
            ok = np.abs(frac - 0.5) > 1e-6
            expect = np.clip(np.floor(ref + 0.5) + 128, 0, 255)
            got = rec[8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
            assert np.array_equal(got[ok], expect[ok])


def pin_inverse_fits_int32_for_any_int16_input(O):
    """With Q <= 4095 every int16 input keeps |S| + 8224 < 2^31 (four
    non-zeros per column of T bound each 1-D pass by 4x)."""
    T = O.T()
    assert ((T != 0).sum(axis=0) == 4).all()
    worst = 0
    for r in range(8):
        for c in range(8):
            sgn = np.outer(T[:, r], T[:, c])
            W = np.where(sgn > 0, 32767 * 4095, np.where(sgn < 0, -32768 * 4095, 0))
            S = O.inverse_block(W)
            worst = max(worst, int(np.abs(S).max()))
    assert worst + 8224 < 2 ** 31


# ---- plane layout ---------------------------------------------------------

def pin_stride_and_block_order(O):
    img = synth.textured(40, 24, 15, stride=56)
    sub = np.ascontiguousarray(img[:, :40])
    Q = synth.qtable(1, 3)
    assert np.array_equal(O.quantise(img, Q, 64, w=40), O.quantise(sub, Q, 64))
    q = O.quantise(sub, Q, 64)
    blk = 7  # by = 1, bx = 2 for w = 40 (5 blocks per row)
    one = np.ascontiguousarray(sub[8:16, 16:24])
    assert np.array_equal(q[blk], O.quantise(one, Q, 64)[0])
    rec = O.inverse(q, Q, 40, 24, dst_stride=48)
    assert np.array_equal(rec[:, :40], O.inverse(q, Q, 40, 24))


def pin_i8_zigzag_is_saturated_scan_of_int16(O):
    img = synth.textured(64, 32, 16)
    Q = synth.qtable(1, 1)
    q16 = O.quantise(img, Q, 64).astype(np.int64)
    q8 = O.quantise_i8_zigzag(img, Q)
    order = O.zigzag_order()
    assert np.array_equal(q8, np.clip(q16[:, order], -128, 127).astype(np.int8))
    assert (np.abs(q16) > 127).any()  # the case actually saturates


def pin_threaded_oracle_equals_single_thread(O):
    img = synth.textured(128, 96, 17)
    Q = synth.qtable(1, 5)
    a = O.quantise(img, Q, 64, threads=1)
    b = O.quantise(img, Q, 64, threads=5)
    assert np.array_equal(a, b)
    assert np.array_equal(O.inverse(a, Q, 128, 96, threads=1),
                          O.inverse(a, Q, 128, 96, threads=3))


PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__[4:])
def test_pin_holds_for_the_oracle(pin, oracle_mod):
    pin(oracle_mod.default())
