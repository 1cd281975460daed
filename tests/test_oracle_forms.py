"""Pins of the oracle's forms (forms_oracle.c) against facts that do not come
from the oracle itself: FP32 rounding bounds around the FP64 iteration, the
closed form for A = I, the one-step hyperplane property, exact integer
arithmetic, numpy's least-squares and projection, and the minimum-norm limit
of Kaczmarz from zero on an underdetermined system (Sec. 2.1)."""
import numpy as np
import pytest

import oracle
from workloads import _round_np, bf16_bits_to_f64

U32 = 2.0 ** -24


def _system(m, n, seed, noise=0.0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)).astype(dtype)
    xs = rng.standard_normal(n)
    b = A.astype(np.float64) @ xs
    if noise:
        b = b + noise * rng.standard_normal(m)
    return A, xs, b


@pytest.mark.parametrize("q,K", [(1, 50), (8, 120), (32, 60)])
def test_rka_f32_tracks_fp64_within_rounding(q, K):
    # same stream, binary32 vs binary64 arithmetic: the gap is rounding only,
    # bounded by K steps of (dot of length n) relative error, and not zero
    A, xs, b = _system(300, 48, 1)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, 5, 0, K, q)
    x32 = oracle.rka_f32_given(A, b, np.zeros(48), idx, q=q)
    x64 = oracle.rka_given(A, b, np.zeros(48), idx, q=q)
    gap = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert 0 < gap <= 4 * K * 48 * U32
    # and the binary32 result is exactly representable in binary32
    assert np.array_equal(x32.astype(np.float32).astype(np.float64), x32)


@pytest.mark.parametrize("q,bs,K", [(1, 5, 20), (4, 10, 15), (16, 3, 10)])
def test_rkab_f32_tracks_fp64_within_rounding(q, bs, K):
    A, xs, b = _system(250, 40, 2)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, 9, 0, K, q, bs)
    x32 = oracle.rkab_f32_given(A, b, np.zeros(40), idx, q=q, block_size=bs)
    x64 = oracle.rkab_given(A, b, np.zeros(40), idx, q=q, block_size=bs)
    gap = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert 0 < gap <= 4 * K * bs * 40 * U32


def test_rka_f32_bf16_storage_matches_widened_f32():
    # bf16 storage widens exactly: running on the bf16 bits or on the same
    # values stored as float32 is the same computation
    rng = np.random.default_rng(3)
    A32 = rng.standard_normal((200, 32)).astype(np.float32)
    bits = _round_np(A32, "bf16")
    Aw = bf16_bits_to_f64(bits).astype(np.float32)
    b = Aw.astype(np.float64) @ rng.standard_normal(32)
    w = oracle.row_norms(bits, dtype="bf16")
    idx = oracle.indices(w, 4, 0, 30, 8)
    xa = oracle.rka_f32_given(bits, b, np.zeros(32), idx, q=8, dtype="bf16")
    xb = oracle.rka_f32_given(Aw, b, np.zeros(32), idx, q=8)
    assert np.array_equal(xa, xb)


def test_rka_f32_identity_closed_form():
    # A = I: x_c <- x_c + (alpha/q) cnt_c (b_c - x_c), cnt_c = workers on row c
    n, q, alpha, K = 16, 6, 0.7, 25
    A = np.eye(n, dtype=np.float32)
    b = np.random.default_rng(4).standard_normal(n)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, 11, 0, K, q)
    x = np.zeros(n)
    for k in range(K):
        cnt = np.bincount(idx[k * q:(k + 1) * q], minlength=n)
        x = x + (alpha / q) * cnt * (b - x)
    x32 = oracle.rka_f32_given(A, b, np.zeros(n), idx, q=q, alpha=alpha)
    assert np.max(np.abs(x32 - x)) <= 8 * K * U32 * np.max(np.abs(b))


def test_rka_f32_one_step_lands_on_hyperplane():
    # q = 1, alpha = 1: x1 is the projection onto H_i (Sec. 2.1), so the
    # sampled row's residual vanishes up to binary32 rounding
    A, _, b = _system(100, 64, 5)
    x0 = np.random.default_rng(6).standard_normal(64).astype(np.float32).astype(np.float64)
    w = oracle.row_norms(A)
    for it in range(5):
        idx = oracle.indices(w, 7, it, 1, 1)
        x1 = oracle.rka_f32_given(A, b, x0, idx, q=1)
        i = idx[0]
        a = A[i].astype(np.float64)
        res = abs(b[i] - a @ x1)
        before = abs(b[i] - a @ x0)
        assert res <= 4 * 64 * U32 * np.linalg.norm(a) * (np.linalg.norm(x1) + abs(b[i]) /
                                                         np.linalg.norm(a))
        assert res < 1e-4 * before


def test_rkab_f32_block1_is_rka_f32_up_to_rounding():
    A, _, b = _system(150, 24, 7)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, 13, 0, 40, 4)
    xa = oracle.rka_f32_given(A, b, np.zeros(24), idx, q=4)
    xb = oracle.rkab_f32_given(A, b, np.zeros(24), idx, q=4, block_size=1)
    assert np.linalg.norm(xa - xb) <= 4 * 40 * 24 * U32 * np.linalg.norm(xa)


def test_transpose_matches_numpy():
    rng = np.random.default_rng(8)
    for dt in (np.float64, np.float32):
        A = rng.standard_normal((37, 23)).astype(dt)
        assert np.array_equal(oracle.transpose(A), A.T)
    bits = _round_np(rng.standard_normal((19, 41)), "bf16")
    assert np.array_equal(oracle.transpose(bits, dtype="bf16"), bits.T)


def test_gemv_exact_on_integers():
    # integer data: every partial sum is exact in binary64
    rng = np.random.default_rng(9)
    M = rng.integers(-50, 50, size=(30, 70)).astype(np.float32)
    v = rng.integers(-50, 50, size=70).astype(np.float64)
    c = rng.integers(-1000, 1000, size=30).astype(np.float64)
    exact = [int(ci) - sum(int(a) * int(x) for a, x in zip(row, v)) for row, ci in zip(M, c)]
    assert np.array_equal(oracle.gemv(M, v, c=c, gamma=-1.0), np.array(exact, dtype=np.float64))
    exact2 = [sum(int(a) * int(x) for a, x in zip(row, v)) for row in M]
    assert np.array_equal(oracle.gemv(M, v), np.array(exact2, dtype=np.float64))


def test_kaczmarz_from_zero_gives_min_norm_projection():
    # the column solve: RKA on A^T y = A^T r from y = 0 tends to the
    # minimum-norm solution, which is the projection of r onto range(A)
    A, _, _ = _system(60, 12, 10, dtype=np.float64)
    r = np.random.default_rng(11).standard_normal(60)
    At = np.ascontiguousarray(A.T)
    g = At @ r
    y, info = oracle.rka(At, g, q=4, alpha=1.0, max_iter=6000, seed=3)
    Q, _ = np.linalg.qr(A)
    proj = Q @ (Q.T @ r)
    assert np.linalg.norm(y - proj) <= 1e-10 * np.linalg.norm(proj)


def test_refine_consistent_reaches_fp64_accuracy():
    # planted consistent system: plain refinement (no range step) with FP32
    # inner solves contracts the error every sweep down to binary64 rounding
    A, xs, b = _system(400, 40, 12)
    x, meas = oracle.refine(A, b, q=8, acc32=1, inner_iters=600, sweeps=5, x_ref=xs)
    assert meas[0] < 1e-3
    assert meas[1] < 1e-3 * meas[0]
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)


@pytest.mark.parametrize("method,bs", [(0, 1), (1, 5)])
def test_refine_inconsistent_reaches_least_squares(method, bs):
    # b = A x* + noise: the range projection removes the least-squares
    # residual from every correction, so the sweeps reach x_LS (numpy) to
    # binary64 accuracy; without it they stall at the horizon
    A, _, b = _system(400, 40, 13, noise=0.1)
    xls = np.linalg.lstsq(A.astype(np.float64), b, rcond=None)[0]
    kw = dict(method=method, q=8, block_size=bs, acc32=1, inner_iters=800 // bs, x_ref=xls)
    x, meas = oracle.refine(A, b, range_iters=800, range_q=8, sweeps=5, **kw)
    assert np.linalg.norm(x - xls) <= 1e-12 * np.linalg.norm(xls)
    _, stall = oracle.refine(A, b, sweeps=4, **kw)
    assert min(stall) > 1e-4


def test_refine_residual_measure_and_fp64_inner():
    # without x_ref the measure is ||b - A x|| / ||b||, which tends to the
    # least-squares residual ratio; FP64 inner solves converge the same way
    A, _, b = _system(300, 30, 14, noise=0.1, dtype=np.float64)
    xls = np.linalg.lstsq(A, b, rcond=None)[0]
    ratio = np.linalg.norm(b - A @ xls) / np.linalg.norm(b)
    x, meas = oracle.refine(A, b, q=8, acc32=0, inner_iters=800, range_iters=800, range_q=8,
                            sweeps=4)
    assert abs(meas[-1] - ratio) <= 1e-12 * ratio
    assert np.linalg.norm(x - xls) <= 1e-12 * np.linalg.norm(xls)
    with pytest.raises(ValueError):  # FP32 accumulation needs narrow storage
        oracle.refine(A, b, q=8, acc32=1, inner_iters=10, sweeps=1)


# -- binary32 operation order, pinned by hand-worked examples -------------------
# Every expected value below is worked out by hand from IEEE binary32
# round-to-nearest-even; each example is built so that another order or
# another precision of the same step gives a different, stated result.
T = 2.0 ** -24  # half an ulp of 1 in binary32: 1 + T rounds to 1 (ties to even)


def test_rka_f32_dot_is_left_to_right_binary32():
    """One RK step (q = 1, alpha = 1) on the row a = (1, 1, 1), b = 3, from
    x = (1, T, T).  Left to right in binary32 the dot is 1 (1 + T rounds down
    to even, twice); the scale is (3 - 1) / 3 = 2/3 rounded, 11184811 * 2^-24;
    then x_0 = 1 + that rounds up to even, 13981014 * 2^-23, and x_1 = x_2 =
    T + s = 11184812 * 2^-24 exactly.  With the dot kept in binary64 (1 + 2T)
    the scale would be 11184810 * 2^-24 and x = (1.6666666269302368,
    0.6666666865348816, 0.6666666865348816)."""
    A = np.ones((1, 3), dtype=np.float32)
    b = np.array([3.0])
    x0 = np.array([1.0, T, T])
    x = oracle.rka_f32_given(A, b, x0, np.zeros(1, dtype=np.int32), q=1)
    assert x[0] == 13981014 * 2.0 ** -23 == 1.6666667461395264
    assert x[1] == x[2] == 11184812 * 2.0 ** -24 == 0.6666667461395264


def test_rka_f32_average_sums_workers_in_order_then_scales():
    """Three workers on three one-column rows (1), b = (1, T, T), from x = 0:
    the scales are b itself; their sum in worker order is 1 + T + T = 1 in
    binary32 (T + T + 1 would be 1 + 2T), times (1/3) rounded to binary32
    (11184811 * 2^-25) gives x = 0.3333333432674408 exactly."""
    A = np.ones((3, 1), dtype=np.float32)
    b = np.array([1.0, T, T])
    x = oracle.rka_f32_given(A, b, np.zeros(1), np.array([0, 1, 2], dtype=np.int32), q=3)
    assert x[0] == 11184811 * 2.0 ** -25 == 0.3333333432674408


def test_rkab_f32_average_divides_the_ordered_sum():
    """The same three rows as RKAB with one projection per worker: the worker
    iterates are (1), (T), (T); their binary32 sum in worker order is 1, and
    1 / 3 rounds to 11184811 * 2^-25."""
    A = np.ones((3, 1), dtype=np.float32)
    b = np.array([1.0, T, T])
    x = oracle.rkab_f32_given(A, b, np.zeros(1), np.array([0, 1, 2], dtype=np.int32), q=3,
                              block_size=1)
    assert x[0] == 11184811 * 2.0 ** -25
    # order matters: the same draws listed with the large one last give
    # T + T + 1 = 1 + 2T, and (1 + 2T) / 3 rounds to 11184812 * 2^-25
    b2 = np.array([T, T, 1.0])
    x2 = oracle.rkab_f32_given(A, b2, np.zeros(1), np.array([0, 1, 2], dtype=np.int32), q=3,
                               block_size=1)
    assert x2[0] == 11184812 * 2.0 ** -25


def test_rka_f32_scale_multiplies_alpha_first():
    """alpha (b - d) / w, evaluated left to right.  alpha = 3, b = 1 and the
    row (1, 1, 1) (w = 3) from x = 0: 3 * 1 / 3 = 1 exactly, so x = (1, 1, 1).
    With b = 0.1 (binary32 13421773 * 2^-27): 3 * b rounds to 10066330 * 2^-25
    and that over 3 rounds back to 13421773 * 2^-27, while alpha times (b / 3)
    would round to 13421774 * 2^-27."""
    A = np.ones((1, 3), dtype=np.float32)
    x = oracle.rka_f32_given(A, np.array([1.0]), np.zeros(3), np.zeros(1, dtype=np.int32), q=1,
                             alpha=3.0)
    assert np.array_equal(x, np.ones(3))
    x = oracle.rka_f32_given(A, np.array([0.1]), np.zeros(3), np.zeros(1, dtype=np.int32), q=1,
                             alpha=3.0)
    b32 = float(np.float32(0.1))
    assert b32 == 13421773 * 2.0 ** -27
    assert np.all(x == 13421773 * 2.0 ** -27)
