"""GPU parity of the precision-form building blocks, through the C ABI:
FP32-accumulation inner solves, the FP64 GEMV / transpose / rank-2 steps, and
the refinement sweeps, each against the oracle on the same seeded inputs.

Bars:
  * transpose: bit-exact;
  * FP64 GEMV: every entry within 2 n u64 sum_j |M_ij v_j| of the oracle's
    (the two sum in different orders; each partial sum errs by at most that);
  * FP32 inner solves (same index stream): norm-wise within the bar of
    tests/bars.py -- 16 times the oracle's own distance between its binary32
    and binary64 iterations on that stream (about 2e-6 here), which one wrong
    row or a doubled weight exceeds by orders of magnitude (tests/test_bars.py);
  * refinement: the final x within 1e-12 of the oracle's refined x, and both
    within 1e-12 of the exact solution (planted x*, or numpy's x_LS).
"""
import numpy as np
import pytest

import oracle
import parity_cases as pc
import workloads
from bars import binary32_bar, oracle_pair, rel
from gpu_util import DEV, assert_x_close, host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


def _system(m, n, dtype, seed=1, noise=0.0):
    A, xs, b = workloads.gaussian_system(m, n, seed=seed, noise_var=noise, dtype=dtype)
    return np.array(A), xs, b


def _odt(dtype):
    return "bf16" if dtype == "bf16" else None


def _widen(A, dtype):
    return workloads.bf16_bits_to_f64(A) if dtype == "bf16" else A.astype(np.float64)


# -- FP32-accumulation inner solves --------------------------------------------

@pytest.mark.parametrize("m,n,q,K,dtype,grid,ar,alpha", pc.RKA32_CASES)
def test_rka_fp32_inner_vs_oracle(m, n, q, K, dtype, grid, ar, alpha):
    say(f"rka fp32 {dtype} {m}x{n} q={q} K={K} grid={grid} ar={ar} alpha={alpha}")
    A, _, b = _system(m, n, dtype, seed=pc.RKA32_SEED_DATA, noise=0.01)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=0, q=q, alpha=alpha, max_iter=K,
                               seed=pc.RKA32_SEED_SOLVE, grid=grid, allreduce=ar, accumulate=1)
    assert info.status == rka.OK and st["accumulate"] == 1 and st["kernel"] == 1
    w = oracle.row_norms(A, dtype=_odt(dtype))
    idx = oracle.indices(w, pc.RKA32_SEED_SOLVE, 0, K, q)
    xo, x64 = oracle_pair(oracle, A, b, np.zeros(n), idx, q=q, alpha=alpha, dtype=_odt(dtype))
    xg = host(x)
    gap, bar = rel(xg, xo), binary32_bar(xo, x64)
    say(f"  gap {gap:.3e}  bar {bar:.3e}")
    assert gap <= bar, (gap, bar)
    # binary32 iterate, widened on the way out
    assert np.array_equal(xg.astype(np.float32).astype(np.float64), xg)


@pytest.mark.parametrize("m,n,q,bs,K,dtype,alpha", pc.RKAB32_CASES)
def test_rkab_fp32_inner_vs_oracle(m, n, q, bs, K, dtype, alpha):
    say(f"rkab fp32 {dtype} {m}x{n} q={q} bs={bs} K={K} alpha={alpha}")
    A, _, b = _system(m, n, dtype, seed=pc.RKAB32_SEED_DATA, noise=0.01)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=1, q=q, block_size=bs,
                               alpha=alpha, max_iter=K, seed=pc.RKAB32_SEED_SOLVE, accumulate=1)
    assert info.status == rka.OK and st["accumulate"] == 1 and st["kernel"] == 2
    w = oracle.row_norms(A, dtype=_odt(dtype))
    idx = oracle.indices(w, pc.RKAB32_SEED_SOLVE, 0, K, q, bs)
    xo, x64 = oracle_pair(oracle, A, b, np.zeros(n), idx, q=q, block_size=bs, alpha=alpha,
                          dtype=_odt(dtype), rkab=True)
    gap, bar = rel(host(x), xo), binary32_bar(xo, x64)
    say(f"  gap {gap:.3e}  bar {bar:.3e}")
    assert gap <= bar, (gap, bar)
    if n == 16000:
        assert st["variant"] == 1  # iterate kept in LDS


def test_fp32_accumulation_needs_narrow_storage():
    A, _, b = _system(50, 8, "f64")
    with pytest.raises(rka.RKAError) as e:
        rka.solve_ex(to_dev(A), vec(b), method=0, q=2, max_iter=3, accumulate=1)
    assert e.value.status == rka.EINVAL


def test_stream_id_selects_the_row_stream():
    # dom = 1 draws the oracle's dom-1 stream (the refinement's column solves)
    A, _, b = _system(500, 64, "f32", seed=7)
    x, info, _ = rka.solve_ex(to_dev(A, "f32"), vec(b), method=0, q=4, max_iter=30, seed=9,
                              accumulate=1, stream_id=1)
    w = oracle.row_norms(A)
    xo, x64 = oracle_pair(oracle, A, b, np.zeros(64), oracle.indices(w, 9, 0, 30, 4, dom=1), q=4)
    assert rel(host(x), xo) <= binary32_bar(xo, x64)


# -- dense steps ---------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("rows,cols", [(1, 1), (5, 7), (513, 1000), (130, 4099), (64, 16)])
def test_gemv_vs_oracle(dtype, rows, cols):
    say(f"gemv {dtype} {rows}x{cols}")
    M, _, _ = _system(rows, cols, dtype, seed=8)
    rng = np.random.default_rng(8)
    v, c = rng.standard_normal(cols), rng.standard_normal(rows)
    y = host(rka.gemv(to_dev(M, dtype), vec(v), c=vec(c), gamma=-1.0))
    yo = oracle.gemv(M, v, c=c, gamma=-1.0, dtype=_odt(dtype))
    bound = 2 * cols * U64 * (np.abs(_widen(M, dtype)) @ np.abs(v)) + 4 * U64 * np.abs(c)
    assert np.all(np.abs(y - yo) <= bound)
    y2 = host(rka.gemv(to_dev(M, dtype), vec(v)))
    yo2 = oracle.gemv(M, v, dtype=_odt(dtype))
    assert np.all(np.abs(y2 - yo2) <= bound)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("m,n", [(1, 1), (63, 65), (200, 130), (64, 64), (1000, 3)])
def test_transpose_bitwise(dtype, m, n):
    say(f"transpose {dtype} {m}x{n}")
    A, _, _ = _system(m, n, dtype, seed=9)
    At = rka.transpose(to_dev(A, dtype))
    got = host(At.view(torch.int16) if dtype == "bf16" else At)
    want = oracle.transpose(A, dtype=_odt(dtype))
    if dtype == "bf16":
        want = want.view(np.int16)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("out", ["f64", "f32"])
def test_lsq_grad_A_vs_numpy(out):
    rng = np.random.default_rng(10)
    m, n = 333, 77
    r, z = rng.standard_normal(m), rng.standard_normal(m)
    lam, x = rng.standard_normal(n), rng.standard_normal(n)
    dA = host(rka.lsq_grad_A(vec(r), vec(lam), vec(z), vec(x),
                             dtype=torch.float64 if out == "f64" else torch.float32))
    want = np.outer(r, lam) - np.outer(z, x)
    scale = np.abs(np.outer(r, lam)) + np.abs(np.outer(z, x))
    u = U64 if out == "f64" else U32
    assert np.all(np.abs(dA - want) <= 4 * u * scale + 1e-300)


# -- refinement ----------------------------------------------------------------

REFINE_CASES = [  # m, n, dtype, method, bs, q, inner, sweeps, noise, range_iters
    (1500, 96, "f32", 0, 1, 8, 2000, 4, 0.0, 0),
    (1500, 96, "bf16", 0, 1, 8, 2000, 4, 0.0, 0),
    (1500, 96, "f32", 1, 8, 8, 500, 4, 0.0, 0),
    (1200, 80, "f32", 0, 1, 8, 2000, 4, 0.01, 2000),
    (1200, 80, "bf16", 1, 5, 8, 400, 4, 0.01, 2000),
    (20000, 512, "f32", 0, 1, 64, 600, 3, 0.0, 0),     # many workgroups, alpha*
]


@pytest.mark.parametrize("m,n,dtype,method,bs,q,inner,sweeps,noise,riters", REFINE_CASES)
def test_refine_vs_oracle(m, n, dtype, method, bs, q, inner, sweeps, noise, riters):
    say(f"refine {dtype} {m}x{n} method={method} bs={bs} q={q} inner={inner} "
        f"sweeps={sweeps} noise={noise} range={riters}")
    A, xs, b = _system(m, n, dtype, seed=11, noise=noise)
    Aw = _widen(A, dtype)
    xt = xs if noise == 0.0 else np.linalg.lstsq(Aw, b, rcond=None)[0]
    alpha = 1.0
    if q == 64:  # Eq. (6) from the extreme singular values
        sv = np.linalg.svd(Aw, compute_uv=False)
        F = np.sum(sv ** 2)
        alpha = rka.alpha_star(sv[-1] ** 2 / F, sv[0] ** 2 / F, q)
    Ad = to_dev(A, dtype)
    At = rka.transpose(Ad) if riters else None
    x, info = rka.refine_solve(Ad, vec(b), At=At, method=method, q=q, block_size=bs,
                               accumulate=1, alpha=alpha, inner_iters=inner, range_iters=riters,
                               range_q=q, max_sweeps=sweeps, seed=13, x_ref=vec(xt))
    xo, mo = oracle.refine(A, b, method=method, q=q, block_size=bs, acc32=1, alpha=alpha,
                           inner_iters=inner, range_iters=riters, range_q=q, sweeps=sweeps,
                           seed=13, x_ref=xt, dtype=_odt(dtype))
    xg = host(x)
    assert info.status == rka.OK and info.sweeps == sweeps
    # the first sweep's measure agrees up to binary32 rounding of the inner
    # solve (relative, or absolute once the inner solve reaches its floor)
    assert abs(info.measures[0] - mo[0]) <= 1e-3 * mo[0] + 1e-5
    assert_x_close(xg, xo, 1e-12, "refined x vs oracle")
    assert_x_close(xg, xt, 1e-12, "refined x vs exact")


def test_refine_stops_at_tol_and_reports_residual():
    A, xs, b = _system(1500, 96, "f32", seed=12)
    x, info = rka.refine_solve(to_dev(A, "f32"), vec(b), q=8, inner_iters=1000, max_sweeps=8,
                               tol=1e-9, seed=2)
    assert info.status == rka.OK and info.sweeps < 8 and info.measures[-1] <= 1e-9
    Aw = A.astype(np.float64)
    res = np.linalg.norm(b - Aw @ host(x)) / np.linalg.norm(b)
    assert abs(res - info.measures[-1]) <= 1e-3 * max(res, 1e-14) + 1e-15


def test_refine_errors():
    A, _, b = _system(100, 10, "f32")
    Ad = to_dev(A, "f32")
    for kw in (dict(range_iters=10), dict(q=0), dict(max_sweeps=0), dict(alpha=-1.0)):
        args = dict(q=2, inner_iters=5, max_sweeps=1)
        args.update(kw)
        with pytest.raises(rka.RKAError) as e:
            rka.refine_solve(Ad, vec(b), **args)
        assert e.value.status == rka.EINVAL
    with pytest.raises(rka.RKAError):  # FP32 accumulation on FP64 storage
        rka.refine_solve(to_dev(A.astype(np.float64)), vec(b), q=2, inner_iters=5,
                         max_sweeps=1, accumulate=1)


def test_refine_inner_solves_stop_at_the_sweep_tolerance():
    # with x_ref and tol, an inner solve ends once ||x + d - x_ref|| <= tol ||x_ref||
    A, xs, b = _system(1500, 96, "f32", seed=14)
    Ad = to_dev(A, "f32")
    x1, full = rka.refine_solve(Ad, vec(b), q=8, inner_iters=3000, max_sweeps=4, seed=4,
                                x_ref=vec(xs))
    x2, early = rka.refine_solve(Ad, vec(b), q=8, inner_iters=3000, max_sweeps=4, seed=4,
                                 x_ref=vec(xs), tol=1e-5)
    assert early.status == rka.OK and early.sweeps == 1 and early.measures[0] <= 1e-5
    assert early.projections < full.projections / 4
    assert early.projections % (25 * 8) == 0
    err = np.linalg.norm(host(x2) - xs) / np.linalg.norm(xs)
    assert abs(err - early.measures[0]) <= 1e-3 * err
