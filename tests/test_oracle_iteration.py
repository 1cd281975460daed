"""Pins of the oracle's RKA / RKAB iterations against facts fixed outside it.

References are to arXiv 2401.17474.  Each test states the fact it checks:

* geometry of one projection (Sec. 2.1: with unit relaxation the new iterate
  lies on the hyperplane of the row used);
* the exact conditional expectation of one RKA step, obtained by enumerating
  every q-tuple of rows with its probability from Eq. (4), equals the
  Landweber step x + (alpha/||A||_F^2) A^T (b - A x) (textbook closed form);
* the exact one-step mean-square error identity behind the optimal weight of
  Eq. (6), again by enumeration, against its SVD form;
* closed forms for A = I (both methods);
* the reductions stated in the paper: q = 1 gives RK (Sec. 3.3.1) and
  block_size = 1 gives RKA (Sec. 3.4.2); and RKAB with one worker is RK run
  over the concatenated stream;
* convergence to a planted solution (consistent) and to the least-squares
  solution within the error horizon (inconsistent; Sec. 2.2 / 2.3.1);
* stopping rule, resume from an iteration offset, argument errors.
"""
import itertools

import numpy as np
import pytest

import workloads


def _tiny(m=4, n=3, seed=0, noise=0.0):
    g = np.random.default_rng(seed)
    A = g.standard_normal((m, n)) * g.uniform(0.5, 2.0, size=(m, 1))
    x = g.standard_normal(n)
    b = A @ x + noise * g.standard_normal(m)
    return A, x, b


def _probs(A):
    w = np.einsum("ij,ij->i", A, A)
    return w / w.sum()


# -- one projection -----------------------------------------------------------

@pytest.mark.parametrize("alpha", [1.0, 0.5, 1.7])
def test_projection_geometry(orc, alpha):
    A, _, b = _tiny(9, 6, seed=1, noise=0.3)
    x0 = np.random.default_rng(2).standard_normal(6)
    for i in range(9):
        x1 = orc.rka_given(A, b, x0, np.array([i]), q=1, alpha=alpha)
        r0 = b[i] - A[i] @ x0
        r1 = b[i] - A[i] @ x1
        scale = np.linalg.norm(A[i]) * max(np.linalg.norm(x1), np.linalg.norm(x0), 1.0)
        assert abs(r1 - (1.0 - alpha) * r0) <= 1e-14 * scale
        # the step is along the row
        d = x1 - x0
        assert np.linalg.norm(d - (d @ A[i]) / (A[i] @ A[i]) * A[i]) <= 1e-14 * scale


def test_rkab_every_inner_projection_hits_its_hyperplane(orc):
    A, _, b = _tiny(7, 5, seed=3, noise=0.2)
    rows = np.array([2, 5, 5, 0])
    v = np.zeros(5)
    for j in range(len(rows)):
        # a one-worker, (j+1)-long block ends exactly after projection j
        v_j = orc.rkab_given(A, b, np.zeros(5), rows[: j + 1], q=1, block_size=j + 1)
        i = rows[j]
        assert abs(b[i] - A[i] @ v_j) <= 1e-13 * np.linalg.norm(A[i]) * np.linalg.norm(v_j)
        v = v_j


# -- exact expectations by enumeration ----------------------------------------

@pytest.mark.parametrize("q,alpha", [(1, 1.0), (2, 1.0), (3, 1.6), (2, 3.1)])
def test_expected_step_is_landweber(orc, q, alpha):
    A, _, b = _tiny(4, 3, seed=4, noise=0.5)
    x = np.array([0.3, -1.2, 0.7])
    p = _probs(A)
    E = np.zeros(3)
    for tup in itertools.product(range(4), repeat=q):
        x1 = orc.rka_given(A, b, x, np.array(tup), q=q, alpha=alpha)
        E += np.prod(p[list(tup)]) * x1
    F = (A * A).sum()
    land = x + alpha / F * A.T @ (b - A @ x)
    assert np.max(np.abs(E - land)) <= 1e-14 * np.linalg.norm(land)


@pytest.mark.parametrize("q,alpha", [(1, 1.0), (2, 1.0), (3, 2.2)])
def test_one_step_error_identity(orc, q, alpha):
    A, _, b = _tiny(5, 3, seed=5, noise=0.8)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    r = b - A @ x_ls
    x = x_ls + np.array([0.5, -0.25, 1.0])
    p = _probs(A)
    E2 = 0.0
    for tup in itertools.product(range(5), repeat=q):
        x1 = orc.rka_given(A, b, x, np.array(tup), q=q, alpha=alpha)
        E2 += np.prod(p[list(tup)]) * np.sum((x1 - x_ls) ** 2)
    F = (A * A).sum()
    _, sig, Vt = np.linalg.svd(A, full_matrices=False)
    s = sig ** 2 / F
    phi = 1 - 2 * alpha * s + alpha ** 2 * s / q + alpha ** 2 * (1 - 1 / q) * s ** 2
    pred = np.sum(phi * (Vt @ (x - x_ls)) ** 2) + alpha ** 2 * (r @ r) / (q * F)
    assert abs(E2 - pred) <= 1e-13 * pred


# -- closed forms for A = I ---------------------------------------------------

def test_identity_closed_form_rka(orc):
    n, q, alpha = 6, 4, 1.3
    A = np.eye(n)
    b = np.arange(1.0, n + 1.0)
    x = np.linspace(-1.0, 1.0, n)
    rows = np.array([0, 3, 3, 5])
    x1 = orc.rka_given(A, b, x, rows, q=q, alpha=alpha)
    cnt = np.bincount(rows, minlength=n)
    assert np.allclose(x1, x + alpha / q * cnt * (b - x), rtol=0, atol=1e-15)


def test_identity_closed_form_rkab(orc):
    n, q, bs, alpha = 5, 3, 4, 0.7
    A = np.eye(n)
    b = np.arange(2.0, n + 2.0)
    x = np.linspace(1.0, -1.0, n)
    rows = np.array([0, 0, 1, 4, 2, 2, 2, 3, 4, 4, 1, 0])
    x1 = orc.rkab_given(A, b, x, rows, q=q, block_size=bs, alpha=alpha)
    ref = np.zeros(n)
    for w in range(q):
        cnt = np.bincount(rows[w * bs:(w + 1) * bs], minlength=n)
        ref += b + (1 - alpha) ** cnt * (x - b)
    assert np.allclose(x1, ref / q, rtol=0, atol=1e-14)


# -- reductions ---------------------------------------------------------------

def test_rkab_block_one_equals_rka(orc):
    A, _, b = workloads.gaussian_system(300, 40, seed=12, noise_var=0.01)
    x_a, ia = orc.rka(A, b, q=6, alpha=1.4, max_iter=200, seed=5)
    x_b, ib = orc.rkab(A, b, q=6, block_size=1, alpha=1.4, max_iter=200, seed=5)
    assert ia["iterations"] == ib["iterations"] == 200
    assert np.linalg.norm(x_a - x_b) <= 1e-14 * np.linalg.norm(x_a)


def test_rkab_one_worker_is_rk_over_concatenated_stream(orc):
    A, _, b = workloads.gaussian_system(200, 30, seed=13, noise_var=0.01)
    w = orc.row_norms(A)
    K, bs = 7, 9
    idx = orc.indices(w, seed=21, iter_offset=0, K=K, q=1, bs=bs)
    x_b = orc.rkab_given(A, b, np.zeros(30), idx, q=1, block_size=bs)
    x_rk = orc.rka_given(A, b, np.zeros(30), idx, q=1)  # K*bs single-row steps
    assert np.linalg.norm(x_b - x_rk) <= 1e-14 * np.linalg.norm(x_rk)
    x_s, _ = orc.rkab(A, b, q=1, block_size=bs, max_iter=K, seed=21)
    assert np.array_equal(x_s, x_b)


def test_rka_one_worker_is_rk(orc):
    A, _, b = workloads.gaussian_system(100, 20, seed=14)
    w = orc.row_norms(A)
    idx = orc.indices(w, seed=2, iter_offset=0, K=50, q=1)
    x_s, _ = orc.rka(A, b, q=1, max_iter=50, seed=2)
    x = np.zeros(20)
    for i in idx:  # Eq. (3) with unit relaxation, rows from the stream
        x = orc.rka_given(A, b, x, np.array([i]), q=1)
    assert np.array_equal(x_s, x)


# -- convergence --------------------------------------------------------------

def test_planted_solution_cfg_small(orc):
    # 4000 x 200 N(0,1), planted x*, q = 8, alpha = 1, tol 1e-8 relative
    A, xs, b = workloads.gaussian_system(4000, 200, seed=workloads.DATA_SEED)
    x, info = orc.rka(A, b, q=8, alpha=1.0, max_iter=200000, tol=1e-8, seed=1, x_ref=xs)
    assert info["status"] == orc.OK
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert 1000 < info["iterations"] < 20000


def test_planted_solution_rkab_and_paper_rows(orc):
    A, xs, b = workloads.paper_rows_system(600, 30, seed=17)
    x, info = orc.rkab(A, b, q=4, block_size=30, alpha=1.0, max_iter=20000, tol=1e-8, seed=3,
                       x_ref=xs)
    assert info["status"] == orc.OK
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)


def test_least_squares_horizon(orc):
    A, _, b = workloads.gaussian_system(400, 20, seed=18, noise_var=0.25)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    # normal equations agree with QR on this well-conditioned system
    assert np.allclose(np.linalg.solve(A.T @ A, A.T @ b), x_ls, rtol=1e-10, atol=1e-12)
    F = (A * A).sum()
    r = b - A @ x_ls
    sig = np.linalg.svd(A, compute_uv=False)
    s = sig ** 2 / F
    errs = {}
    for q in (1, 16):
        e2 = []
        for seed in range(1, 41):
            x, _ = orc.rka(A, b, q=q, alpha=1.0, max_iter=3000, seed=seed)
            e2.append(np.sum((x - x_ls) ** 2))
        phi = 1 - 2 * s + s / q + (1 - 1 / q) * s ** 2
        bound = (r @ r) / (q * F * (1 - phi.max()))
        errs[q] = np.mean(e2)
        assert errs[q] <= 1.5 * bound  # mean over 40 seeds vs the stationary bound
    assert errs[16] < errs[1] / 4      # the horizon shrinks with q (Sec. 3.5)


# -- stopping, resume, errors -------------------------------------------------

def test_stopping_rule_granularity(orc):
    A, xs, b = workloads.gaussian_system(500, 25, seed=19)
    C = 7
    x, info = orc.rka(A, b, q=3, max_iter=100000, tol=1e-6, seed=4, x_ref=xs, check_every=C)
    k = info["iterations"]
    assert info["status"] == orc.OK and k % C == 0
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    xp, _ = orc.rka(A, b, q=3, max_iter=k - C, tol=0.0, seed=4)
    assert np.linalg.norm(xp - xs) > 1e-6 * np.linalg.norm(xs)


def test_residual_stopping_without_reference(orc):
    A, xs, b = workloads.gaussian_system(300, 20, seed=20)
    x, info = orc.rka(A, b, q=2, max_iter=100000, tol=1e-7, seed=4, check_every=10)
    assert info["status"] == orc.OK
    assert np.linalg.norm(b - A @ x) <= 1e-7 * np.linalg.norm(b)


@pytest.mark.parametrize("block", [1, 5])
def test_resume_from_offset(orc, block):
    A, _, b = workloads.gaussian_system(250, 30, seed=21, noise_var=0.1)
    solve = (lambda **kw: orc.rka(A, b, q=4, **kw)) if block == 1 else \
        (lambda **kw: orc.rkab(A, b, q=4, block_size=block, **kw))
    x_full, _ = solve(max_iter=40, seed=8)
    x_half, _ = solve(max_iter=15, seed=8)
    x_rest, _ = solve(max_iter=25, seed=8, x0=x_half, iter_offset=15)
    assert np.array_equal(x_full, x_rest)


def test_narrow_storage_equals_widened(orc):
    for dt in ("f32", "bf16"):
        A, _, b = workloads.gaussian_system(120, 17, seed=22, dtype=dt)
        Ad = workloads._widen_np(A, dt)
        x1, _ = orc.rkab(A, b, q=3, block_size=4, max_iter=30, seed=2,
                         dtype="bf16" if dt == "bf16" else None)
        x2, _ = orc.rkab(Ad, b, q=3, block_size=4, max_iter=30, seed=2)
        assert np.array_equal(x1, x2)


def test_errors(orc):
    A, _, b = workloads.gaussian_system(20, 5, seed=23)
    _, info = orc.rka(A, b, q=0, max_iter=3)
    assert info["status"] == orc.EINVAL
    _, info = orc.rka(A, b, q=2, alpha=0.0, max_iter=3)
    assert info["status"] == orc.EINVAL
    bad = b.copy()
    bad[3] = np.nan
    _, info = orc.rka(A, bad, q=2, max_iter=3)
    assert info["status"] == orc.EINVAL
    _, info = orc.rka(np.zeros((4, 3)), np.zeros(4), q=2, max_iter=3)
    assert info["status"] == orc.EZERONORM
    # a huge relaxation with duplicated rows diverges and is reported as such
    Ad = np.vstack([A, A])
    bd = np.concatenate([b, b + 1.0])
    _, info = orc.rka(Ad, bd, q=1, alpha=50.0, max_iter=2000, tol=1e-12, seed=1,
                      check_every=50)
    assert info["status"] == orc.EDIVERGED
