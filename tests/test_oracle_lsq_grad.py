"""Pins of the least-squares gradient oracle (oracle/lsq_grad.py): central
finite differences of the least-squares map computed by a different routine
(numpy's SVD-based lstsq), and the algebraic identities of the adjoint."""
import numpy as np
import pytest

import workloads
from oracle.lsq_grad import lsq, lsq_grad


def _problem(m=200, n=20, seed=5):
    A, xs, b = workloads.gaussian_system(m, n, seed=seed, noise_var=1e-2)
    t = np.random.default_rng(seed + 1).standard_normal(n)
    return np.array(A), b, t


def _loss(A, b, t):
    x = np.linalg.lstsq(A, b, rcond=None)[0]
    return float(np.sum((x - t) ** 2))


def test_solution_matches_lstsq():
    A, b, _ = _problem()
    assert np.allclose(lsq(A, b), np.linalg.lstsq(A, b, rcond=None)[0], rtol=1e-13, atol=1e-14)


def test_gradient_matches_central_differences():
    # L = ||x(A, b) - t||^2, dL/dx = 2 (x - t)
    A, b, t = _problem()
    x = lsq(A, b)
    _, _, _, _, dA, db = lsq_grad(A, b, 2.0 * (x - t))
    rng = np.random.default_rng(7)
    h = 1e-6
    for _ in range(25):
        i, j = rng.integers(0, A.shape[0]), rng.integers(0, A.shape[1])
        Ap, Am = A.copy(), A.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (_loss(Ap, b, t) - _loss(Am, b, t)) / (2 * h)
        assert abs(fd - dA[i, j]) <= 1e-6 * max(1.0, abs(dA[i, j])), (i, j, fd, dA[i, j])
    for _ in range(10):
        i = rng.integers(0, A.shape[0])
        bp, bm = b.copy(), b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (_loss(A, bp, t) - _loss(A, bm, t)) / (2 * h)
        assert abs(fd - db[i]) <= 1e-6 * max(1.0, abs(db[i]))


def test_adjoint_identities():
    A, b, t = _problem(300, 30, 9)
    g = np.random.default_rng(3).standard_normal(30)
    x, r, lam, z, dA, db = lsq_grad(A, b, g)
    assert np.allclose(A.T @ z, g, rtol=0, atol=1e-12 * np.linalg.norm(g))      # A^T z = g
    assert np.linalg.norm(A.T @ r) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(r)
    # z is the minimum-norm solution: it lies in range(A)
    Q, _ = np.linalg.qr(A)
    assert np.linalg.norm(z - Q @ (Q.T @ z)) <= 1e-12 * np.linalg.norm(z)
    assert np.allclose(A @ lam, z, rtol=0, atol=1e-12 * np.linalg.norm(z))
    # the gradient is linear in g: a planted mistake in a sign shows here too
    _, _, lam2, z2, dA2, _ = lsq_grad(A, b, 2 * g)
    assert np.allclose(dA2, 2 * dA, rtol=1e-12, atol=1e-14)
