"""Pins of the oracle's Distributed Approach and per-worker weights
(Sec. 3.3.2): block containment, reduction to the full-matrix stream at q = 1,
the within-block distribution (chi-square), equal weights reducing to the
scalar-weight iterations, and convergence of both variants on a planted
system."""
import numpy as np
import pytest
from scipy import stats

import oracle
import workloads


def _w(m, seed):
    A, _, _ = workloads.gaussian_system(m, 8, seed=seed)
    return oracle.row_norms(np.array(A) * np.linspace(0.2, 3.0, m)[:, None])


def test_every_draw_stays_in_its_workers_block():
    m, q, bs, K = 103, 7, 3, 40
    idx = oracle.indices_blocks(_w(m, 1), 5, 0, K, q, bs).reshape(K, q, bs)
    for w in range(q):
        lo, hi = w * m // q, (w + 1) * m // q
        assert np.all((idx[:, w, :] >= lo) & (idx[:, w, :] < hi))


def test_one_worker_is_the_full_matrix_stream():
    w = _w(500, 2)
    assert np.array_equal(oracle.indices_blocks(w, 9, 3, 50, 1, 4),
                          oracle.indices(w, 9, 3, 50, 1, 4))


def test_within_block_distribution_follows_the_norms():
    m, q = 60, 3
    w = _w(m, 3)
    idx = oracle.indices_blocks(w, 11, 0, 20000, q, 1).reshape(-1, q)
    for wk in range(q):
        lo, hi = wk * m // q, (wk + 1) * m // q
        counts = np.bincount(idx[:, wk] - lo, minlength=hi - lo)
        p = w[lo:hi] / w[lo:hi].sum()
        chi2 = np.sum((counts - 20000 * p) ** 2 / (20000 * p))
        assert stats.chi2.sf(chi2, hi - lo - 1) > 1e-4


def test_zero_weight_block_is_an_error():
    w = _w(40, 4)
    w[10:20] = 0.0  # the second of four blocks
    with pytest.raises(ValueError):
        oracle.indices_blocks(w, 1, 0, 5, 4)


@pytest.mark.parametrize("q,bs", [(1, 1), (6, 1), (5, 4)])
def test_equal_worker_weights_are_the_scalar_weight_iteration(q, bs):
    A, _, b = workloads.gaussian_system(300, 20, seed=5, noise_var=1e-2)
    A = np.array(A)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, 7, 0, 30, q, bs)
    wa = np.full(q, 0.9)
    if bs == 1:
        xa = oracle.rka_walpha_given(A, b, np.zeros(20), idx, wa, q=q)
        xb = oracle.rka_given(A, b, np.zeros(20), idx, q=q, alpha=0.9)
    else:
        xa = oracle.rkab_walpha_given(A, b, np.zeros(20), idx, wa, q=q, block_size=bs)
        xb = oracle.rkab_given(A, b, np.zeros(20), idx, q=q, block_size=bs, alpha=0.9)
    assert np.linalg.norm(xa - xb) <= 1e-13 * np.linalg.norm(xb)


def test_distinct_weights_change_each_workers_step():
    # one worker with weight 0 contributes nothing: with q = 2 the average is
    # half of worker 1's projection step
    A, _, b = workloads.gaussian_system(200, 10, seed=6)
    A = np.array(A)
    idx = oracle.indices(oracle.row_norms(A), 8, 0, 1, 2)
    x = oracle.rka_walpha_given(A, b, np.zeros(10), idx, np.array([0.0, 1.0]), q=2)
    i = idx[1]
    step = (b[i] / np.dot(A[i], A[i])) * A[i]
    assert np.allclose(x, 0.5 * step, rtol=1e-14, atol=1e-15)


def test_distributed_approach_converges_on_a_planted_system():
    A, xs, b = workloads.gaussian_system(2000, 50, seed=7)
    A = np.array(A)
    w = oracle.row_norms(A)
    q, K = 8, 3000
    x = oracle.rka_walpha_given(A, b, np.zeros(50), oracle.indices_blocks(w, 3, 0, K, q),
                                np.full(q, 1.0), q=q)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
