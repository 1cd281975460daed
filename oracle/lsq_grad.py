"""Least-squares solution and its gradient, from their definitions, in FP64 --
TEST INFRASTRUCTURE ONLY (the oracle of the differentiable solve).

For A (m x n, full column rank) and b, x(A, b) = argmin ||A x - b|| (the
problem of Eq. (2) of arXiv 2401.17474 in the inconsistent case).  For a loss
L(x) with g = dL/dx, differentiating the normal equations A^T A x = A^T b
gives, with r = b - A x and lambda = (A^T A)^{-1} g,

    dL/db = z = A lambda        (the minimum-norm solution of A^T z = g)
    dL/dA = r lambda^T - z x^T

Everything goes through one reduced QR factorisation A = Q R (so A^T A =
R^T R): x = R^{-1} Q^T b and lambda = R^{-1} R^{-T} g.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _qr(A):
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="reduced")
    return Q, R


def lsq(A, b):
    """x = argmin ||A x - b|| by QR."""
    Q, R = _qr(A)
    return sla.solve_triangular(R, Q.T @ np.asarray(b, dtype=np.float64))


def lsq_grad(A, b, g):
    """(x, r, lambda, z, dA, db) for upstream gradient g = dL/dx."""
    A = np.asarray(A, dtype=np.float64)
    Q, R = _qr(A)
    x = sla.solve_triangular(R, Q.T @ b)
    r = b - A @ x
    lam = sla.solve_triangular(R, sla.solve_triangular(R, g, trans="T"))
    z = A @ lam
    dA = np.outer(r, lam) - np.outer(z, x)
    return x, r, lam, z, dA, z.copy()
