"""Pins of the oracle's cyclic order (Sec. 2.1) and row weights (Eq. (7)).

References are to arXiv 2401.17474.  Each test states the fact it checks:

* a hand-worked 2 x 2 run of Cyclic Kaczmarz (four projections computed on
  paper below), which fixes the order of the rows and the arithmetic;
* rows that are mutually orthogonal: one sweep of CK with unit relaxation
  solves the system exactly (each projection leaves the earlier rows' residuals
  untouched), whatever the row scales;
* an underdetermined consistent system from x = 0 converges to the
  minimum-norm solution (Sec. 2.1), against numpy's pseudo-inverse;
* one projection with relaxation w multiplies the used row's residual by
  (1 - w) (Sec. 2.1 geometry), for CK and for the per-row weighted RKA;
* uniform row weights w_i = alpha reproduce the pinned RKA / RKAB iterations;
* the cyclic index stream is the position of the draw modulo m, and one
  worker running it through the weighted RKA / RKAB is CK;
* a zero row is a step that leaves the iterate unchanged.
"""
import numpy as np
import pytest

import workloads


def test_ck_hand_worked_2x2(orc):
    # A = [[1, 0], [1, 1]], b = [1, 2], x* = (1, 1), x0 = 0:
    #   row 0: r = 1,    x = (1, 0)
    #   row 1: r = 1,    x = (1, 0) + 1/2 (1, 1)     = (1.5, 0.5)
    #   row 0: r = -0.5, x = (1.5, 0.5) - 0.5 (1, 0) = (1, 0.5)
    #   row 1: r = 0.5,  x = (1, 0.5) + 1/4 (1, 1)   = (1.25, 0.75)
    # (starting with row 1 instead would land on x* at once)
    A = np.array([[1.0, 0.0], [1.0, 1.0]])
    b = np.array([1.0, 2.0])
    want = [(1.0, 0.0), (1.5, 0.5), (1.0, 0.5), (1.25, 0.75)]
    for k, w in enumerate(want, start=1):
        np.testing.assert_array_equal(orc.ck(A, b, iters=k), w)


def test_ck_orthogonal_rows_one_sweep_is_exact(orc):
    g = np.random.default_rng(5)
    Q, _ = np.linalg.qr(g.standard_normal((9, 9)))
    A = Q * g.uniform(0.2, 7.0, size=(9, 1))  # orthogonal rows of mixed length
    x = g.standard_normal(9)
    b = A @ x
    got = orc.ck(A, b, iters=9)
    assert np.max(np.abs(got - x)) <= 1e-12 * np.max(np.abs(x)) * 10
    # one row short of a sweep leaves the last row's residual untouched
    part = orc.ck(A, b, iters=8)
    assert abs(b[8] - A[8] @ part) > 1e-3


def test_ck_underdetermined_reaches_min_norm(orc):
    g = np.random.default_rng(6)
    A = g.standard_normal((5, 12))
    b = g.standard_normal(5)
    got = orc.ck(A, b, iters=5 * 400)
    want = np.linalg.pinv(A) @ b
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


@pytest.mark.parametrize("w", [1.0, 0.5, 1.7])
def test_relaxed_step_scales_the_row_residual(orc, w):
    g = np.random.default_rng(7)
    A = g.standard_normal((6, 4)) * g.uniform(0.5, 3.0, size=(6, 1))
    b = g.standard_normal(6)
    x0 = g.standard_normal(4)
    relax = np.full(6, 2.0)  # other rows' relaxations must not matter
    relax[0] = w
    r0 = b[0] - A[0] @ x0
    x1 = orc.ck(A, b, iters=1, relax=relax, x0=x0)
    assert abs((b[0] - A[0] @ x1) - (1.0 - w) * r0) <= 1e-13 * (1 + abs(r0))
    # the weighted RKA with one worker takes the same step through row 3
    wrow = np.full(6, 0.3)
    wrow[3] = w
    r3 = b[3] - A[3] @ x0
    x2 = orc.rka_wrow_given(A, b, x0, np.array([3], np.int32), wrow, q=1)
    assert abs((b[3] - A[3] @ x2) - (1.0 - w) * r3) <= 1e-13 * (1 + abs(r3))


def test_uniform_row_weights_are_rka_and_rkab(orc):
    A, _, b = workloads.paper_rows_system(300, 12, seed=8)
    w = orc.row_norms(A)
    idx = orc.indices(w, 4, 0, 30, 5)
    wrow = np.full(300, 1.3)
    x0 = np.zeros(12)
    got = orc.rka_wrow_given(A, b, x0, idx, wrow, q=5)
    want = orc.rka_given(A, b, x0, idx, q=5, alpha=1.3)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    idxb = orc.indices(w, 4, 0, 10, 3, 4)
    got = orc.rkab_wrow_given(A, b, x0, idxb, wrow, q=3, block_size=4)
    want = orc.rkab_given(A, b, x0, idxb, q=3, block_size=4, alpha=1.3)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_cyclic_indices_are_stream_positions(orc):
    m, off, K, q, bs = 7, 3, 4, 2, 3
    idx = orc.indices_cyclic(m, off, K, q, bs)
    assert idx.shape == (K * q * bs,)
    for k in range(K):
        for w in range(q):
            for j in range(bs):
                assert idx[(k * q + w) * bs + j] == (((k + off) * q + w) * bs + j) % m
    np.testing.assert_array_equal(orc.indices_cyclic(4, 0, 6, 1, 1), [0, 1, 2, 3, 0, 1])


def test_one_worker_on_the_cyclic_stream_is_ck(orc):
    A, _, b = workloads.paper_rows_system(40, 6, seed=9)
    relax = np.random.default_rng(9).uniform(0.4, 1.6, size=40)
    want = orc.ck(A, b, iters=100, relax=relax)
    got = orc.rka_wrow_given(A, b, np.zeros(6), orc.indices_cyclic(40, 0, 100, 1, 1), relax, q=1)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    got = orc.rkab_wrow_given(A, b, np.zeros(6), orc.indices_cyclic(40, 0, 4, 1, 25), relax, q=1,
                              block_size=25)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_zero_row_leaves_the_iterate(orc):
    g = np.random.default_rng(10)
    A = g.standard_normal((5, 3))
    A[2] = 0.0
    b = g.standard_normal(5)
    b[2] = 4.0  # unsatisfiable row: skipped, not divided by zero
    x0 = g.standard_normal(3)
    x = orc.ck(A, b, iters=3, x0=orc.ck(A, b, iters=2, x0=x0))
    np.testing.assert_array_equal(orc.ck(A, b, iters=2, x0=x0), orc.ck(A, b, iters=3, x0=x0))
    assert np.all(np.isfinite(x))
    got = orc.rka_wrow_given(A, b, x0, np.array([2, 2], np.int32), np.ones(5), q=2)
    np.testing.assert_array_equal(got, x0)


def test_coherent_order_permutes_the_rows():
    A1, x1, b1 = workloads.paper_rows_system(200, 7, seed=11)
    A2, x2, b2 = workloads.paper_rows_system(200, 7, seed=11, order="coherent")
    np.testing.assert_array_equal(x1, x2)
    p = np.lexsort(A1.T[::-1])
    r = np.lexsort(A2.T[::-1])
    np.testing.assert_array_equal(A1[p], A2[r])
    np.testing.assert_allclose(A2 @ x2, b2, rtol=0, atol=1e-9 * np.max(np.abs(b2)))
    # neighbours are more nearly parallel than in the drawn order
    def mean_cos(A):
        U = A / np.linalg.norm(A, axis=1, keepdims=True)
        return np.mean(np.abs(np.sum(U[1:] * U[:-1], axis=1)))
    assert mean_cos(A2) > mean_cos(A1)
