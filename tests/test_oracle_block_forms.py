"""The block forms the GPU kernels use, checked against the oracle's
sequential iterations (arXiv 2401.17474).

Neither form is in the paper; both are Eq. (7) and RKAB (Sec. 3.4.1)
unrolled, and are exact in exact arithmetic:

* RKA over a block of p iterations whose rows are drawn ahead: the scales
  s_r = alpha_r (b_r - <a_r, x^(k+j)>) / ||a_r||^2 of iteration j solve
  (I + N) s = c with c_r = alpha_r (b_r - <a_r, x^(k)>) / ||a_r||^2 and
  N_{r,c} = alpha_r <a_r, a_c> / (q ||a_r||^2) for rows c of earlier
  iterations, and x^(k+p) = x^(k) + (1/q) sum_r s_r a_r;
* RKAB, one outer iteration: worker w's scales solve (I + N_w) s_w = c_w with
  N_w[j][l] = alpha_j <a_j, a_l> / ||a_j||^2 for its own earlier rows
  (weight 1), and x^(k+1) = x^(k) + (1/q) sum_w sum_j s_{w,j} a_{w,j}.

Here both are written with dense numpy solves and compared with the oracle
on the same rows (within 1e-12), and a mistake in either (the 1/q in N
dropped, the worker blocks not separated) fails.
"""
import numpy as np
import pytest

import workloads


def _system(m, n, seed):
    A, _, b = workloads.gaussian_system(m, n, seed=seed, noise_var=0.01)
    return np.array(A, dtype=np.float64), np.array(b, dtype=np.float64)


def _rka_block(A, b, x, rows, q, alpha, one_over_q_in_n=True):
    """x after the len(rows) / q iterations of one block (rows iteration-major)."""
    R = rows.size
    a = A[rows]
    w = np.einsum("ij,ij->i", a, a)
    c = alpha * (b[rows] - a @ x) / w
    it = np.arange(R) // q
    G = a @ a.T
    N = np.where(it[:, None] > it[None, :], G, 0.0) * (alpha / w)[:, None]
    if one_over_q_in_n:
        N /= q
    s = np.linalg.solve(np.eye(R) + N, c)
    return x + (s @ a) / q


def _rkab_outer(A, b, x, rows, q, bs, alpha, separate_workers=True):
    """x after one RKAB outer iteration (rows worker-major, bs per worker)."""
    R = rows.size
    a = A[rows]
    w = np.einsum("ij,ij->i", a, a)
    c = alpha * (b[rows] - a @ x) / w
    wk, j = np.arange(R) // bs, np.arange(R) % bs
    same = wk[:, None] == wk[None, :] if separate_workers else np.ones((R, R), bool)
    N = np.where(same & (j[:, None] > j[None, :]), a @ a.T, 0.0) * (alpha / w)[:, None]
    s = np.linalg.solve(np.eye(R) + N, c)
    return x + (s @ a) / q


@pytest.mark.parametrize("q,p,alpha", [(4, 3, 1.0), (8, 5, 1.3), (1, 6, 0.8), (16, 2, 2.0)])
def test_rka_block_form_equals_the_iterations(orc, q, p, alpha):
    A, b = _system(300, 40, seed=q + p)
    rng = np.random.default_rng(q * 7 + p)
    x0 = rng.standard_normal(40)
    rows = rng.integers(0, 300, size=q * p).astype(np.int32)
    ref = orc.rka_given(A, b, x0, rows, q=q, alpha=alpha)
    got = _rka_block(A, b, x0, rows, q, alpha)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    if q > 1:  # the 1/q in N is what makes the block the averaged iteration
        bad = _rka_block(A, b, x0, rows, q, alpha, one_over_q_in_n=False)
        assert np.linalg.norm(bad - ref) > 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("q,bs,alpha", [(4, 3, 1.0), (8, 10, 0.9), (3, 12, 1.2), (16, 2, 1.0)])
def test_rkab_block_form_equals_the_outer_iteration(orc, q, bs, alpha):
    A, b = _system(400, 60, seed=q + bs)
    rng = np.random.default_rng(q * 11 + bs)
    x0 = rng.standard_normal(60)
    rows = rng.integers(0, 400, size=q * bs).astype(np.int32)
    ref = orc.rkab_given(A, b, x0, rows, q=q, block_size=bs, alpha=alpha)
    got = _rkab_outer(A, b, x0, rows, q, bs, alpha)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    if q > 1:  # the workers' blocks are independent: coupling them is wrong
        bad = _rkab_outer(A, b, x0, rows, q, bs, alpha, separate_workers=False)
        assert np.linalg.norm(bad - ref) > 1e-6 * np.linalg.norm(ref)
