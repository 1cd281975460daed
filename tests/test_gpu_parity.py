"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Bars (arXiv 2401.17474 method; tolerances as stated below):
  * row norms, running sum and the sampled row stream: bit-exact;
  * x in FP64: norm-wise relative difference <= 1e-12 and every element within
    1e-12 of the oracle's largest entry, for the same index stream.
Sizes span several tiles / workgroups with ragged tails, and both the 16-byte
vector path and the scalar path (odd n or unaligned pitch).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import DEV, assert_x_close, host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


def _system(m, n, dtype="f64", seed=1, noise=0.01, zero_rows=()):
    A, xs, b = workloads.gaussian_system(m, n, seed=seed, noise_var=noise, dtype=dtype)
    A = np.array(A)
    for r in zero_rows:
        A[r] = 0
    return A, xs, b


# -- sampler side: bit-exact ---------------------------------------------------

NORM_CASES = [(1, 1), (7, 3), (300, 129), (513, 1000), (1000, 2048), (257, 4)]


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("m,n", NORM_CASES)
def test_row_norms_bitwise(dtype, m, n):
    say(f"row_norms {dtype} {m}x{n}")
    A, _, _ = _system(m, n, dtype)
    w = host(rka.row_norms(to_dev(A, dtype)))
    wo = oracle.row_norms(A, dtype="bf16" if dtype == "bf16" else None)
    assert np.array_equal(w, wo)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_row_norms_strided_and_unaligned(dtype):
    say(f"row_norms strided {dtype}")
    A, _, _ = _system(130, 77, dtype)
    Ad = to_dev(A, dtype)
    wo = oracle.row_norms(A, dtype="bf16" if dtype == "bf16" else None)
    # odd pitch (scalar path)
    big = torch.zeros((130, 79), dtype=Ad.dtype, device=DEV)
    big[:, :77] = Ad
    assert np.array_equal(host(rka.row_norms(big[:, :77])), wo)
    # base pointer off 16-byte alignment (scalar path)
    flat = torch.zeros(130 * 80 + 1, dtype=Ad.dtype, device=DEV)
    view = flat[1:].view(130, 80)
    view[:, :77] = Ad
    assert np.array_equal(host(rka.row_norms(view[:, :77])), wo)


@pytest.mark.parametrize("m", [1, 5, 1024, 1025, 5000])
def test_prefix_bitwise(m):
    say(f"prefix m={m}")
    g = np.random.default_rng(m)
    w = g.exponential(size=m) * 10.0 ** g.uniform(-3, 3, size=m)
    w[g.integers(0, m, size=m // 7)] = 0.0
    if m > 1:
        w[-1] = 0.0
    if w.sum() == 0:
        w[0] = 1.0
    c, last = rka.prefix(vec(w))
    co, st = oracle.prefix(w)
    assert st == oracle.OK
    assert np.array_equal(host(c), co)
    assert int(host(last)[0]) == int(np.nonzero(w > 0)[0].max())


def test_prefix_zero_total():
    with pytest.raises(rka.RKAError) as e:
        rka.prefix(vec(np.zeros(10)))
    assert e.value.status == rka.EZERONORM


@pytest.mark.parametrize("m,n,seed,off,K,q,bs,dom", [
    (300, 20, 1, 0, 50, 8, 1, 0),
    (300, 20, 7, 123, 20, 16, 10, 0),
    (4097, 33, 2**40 + 5, 2**33, 5, 64, 3, 0),
    (1000, 10, 9, 0, 7, 300, 2, 1),
])
def test_sample_indices_bitwise(m, n, seed, off, K, q, bs, dom):
    say(f"sample m={m} q={q} bs={bs} off={off} dom={dom}")
    A, _, _ = _system(m, n, zero_rows=range(0, m, 11))
    Ad = to_dev(A)
    w = rka.row_norms(Ad)
    c, _ = rka.prefix(w)
    idx = host(rka.sample_indices(w, c, seed=seed, iter_offset=off, K=K, q=q, bs=bs, dom=dom))
    io = oracle.indices(oracle.row_norms(A), seed=seed, iter_offset=off, K=K, q=q, bs=bs, dom=dom)
    assert np.array_equal(idx, io)
    assert not np.any(np.isin(idx, np.arange(0, m, 11)))  # zero rows never drawn


# -- iterations: FP64 within 1e-12 ----------------------------------------------

RKA_CASES = [
    # m, n, dtype, q, K, alpha      (comment: geometry exercised)
    (700, 48, "f64", 8, 60, 1.0),       # one workgroup
    (700, 47, "f64", 8, 60, 1.3),       # odd n: scalar path
    (2000, 1000, "f64", 16, 40, 1.0),   # grid of column slices, 1 row per thread
    (3000, 1024, "f64", 64, 25, 2.0),   # 4 rows per thread
    (3000, 1536, "f64", 256, 10, 1.0),  # two-barrier exchange
    (2500, 999, "f64", 24, 30, 1.0),    # grid, scalar path, ragged last slice
    (1500, 400, "f32", 16, 40, 1.0),
    (1500, 640, "bf16", 12, 40, 1.0),
    (2000, 3, "f64", 5, 100, 1.0),      # n smaller than a vec
]


@pytest.mark.parametrize("m,n,dtype,q,K,alpha", RKA_CASES)
def test_rka_parity(m, n, dtype, q, K, alpha):
    say(f"rka {dtype} {m}x{n} q={q} K={K}")
    A, _, b = _system(m, n, dtype, seed=m + n)
    x, info = rka.rka_solve(to_dev(A, dtype), vec(b), q=q, alpha=alpha, max_iter=K, seed=11)
    xo, io = oracle.rka(A, b, q=q, alpha=alpha, max_iter=K, seed=11,
                        dtype="bf16" if dtype == "bf16" else None)
    assert info.status == rka.OK and info.iterations == K == io["iterations"]
    assert info.projections == K * q
    assert_x_close(host(x), xo, what=f"rka {m}x{n} q={q}")


RKAB_CASES = [
    (700, 48, "f64", 8, 4, 20, 1.0),
    (2000, 1000, "f64", 16, 10, 8, 1.0),
    (3000, 513, "f64", 300, 2, 4, 1.0),   # more workers than workgroups
    (1500, 200, "f64", 4, 200, 3, 1.0),   # block size = n (the paper's rule of thumb)
    (1500, 640, "f32", 16, 5, 10, 1.2),
    (1500, 640, "bf16", 16, 5, 10, 1.0),
    (900, 101, "f64", 6, 3, 15, 0.8),     # scalar path
    (1200, 8000, "f64", 8, 7, 3, 1.0),    # long rows: worker iterate kept in LDS
    (600, 5001, "f64", 3, 4, 2, 1.0),     # long odd rows: scalar path, registers
]


@pytest.mark.parametrize("m,n,dtype,q,bs,K,alpha", RKAB_CASES)
def test_rkab_parity(m, n, dtype, q, bs, K, alpha):
    say(f"rkab {dtype} {m}x{n} q={q} bs={bs} K={K}")
    A, _, b = _system(m, n, dtype, seed=m + 2 * n)
    x, info = rka.rkab_solve(to_dev(A, dtype), vec(b), q=q, block_size=bs, alpha=alpha,
                             max_iter=K, seed=5)
    xo, io = oracle.rkab(A, b, q=q, block_size=bs, alpha=alpha, max_iter=K, seed=5,
                         dtype="bf16" if dtype == "bf16" else None)
    assert info.status == rka.OK and info.iterations == K
    assert info.projections == K * q * bs
    assert_x_close(host(x), xo, what=f"rkab {m}x{n} q={q} bs={bs}")


@pytest.mark.parametrize("m,n,dtype,q,bs,K,alpha", RKAB_CASES)
def test_rkab_worker_kernel_parity(m, n, dtype, q, bs, K, alpha):
    """The worker-split kernel on the same cases (the library may pick the
    column-split kernel for them by default)."""
    say(f"rkab worker-split {dtype} {m}x{n} q={q} bs={bs} K={K}")
    A, _, b = _system(m, n, dtype, seed=m + 2 * n)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=1, q=q, block_size=bs,
                               alpha=alpha, max_iter=K, seed=5, rkab_split=1)
    assert info.status == rka.OK and st["kernel"] == 2
    xo, _ = oracle.rkab(A, b, q=q, block_size=bs, alpha=alpha, max_iter=K, seed=5,
                        dtype="bf16" if dtype == "bf16" else None)
    assert_x_close(host(x), xo, what=f"rkab worker-split {m}x{n} q={q} bs={bs}")


@pytest.mark.parametrize("q,grid,allreduce", [
    (16, 8, 1), (16, 0, 2), (16, 7, 1), (16, 64, 2), (64, 24, 1), (64, 0, 2), (100, 16, 1),
    (200, 25, 2), (5, 2, 0),
])
def test_rka_allreduce_modes_and_grids(q, grid, allreduce):
    """Every exchange mode and launch geometry reaches the oracle's iterate."""
    say(f"rka modes q={q} grid={grid} allreduce={allreduce}")
    A, _, b = _system(2500, 1200, seed=q + grid)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=q, max_iter=30, seed=9,
                               grid=grid, allreduce=allreduce, steps_per_exchange=1)
    xo, _ = oracle.rka(A, b, q=q, max_iter=30, seed=9)
    assert info.status == rka.OK and st["kernel"] == 1
    if grid:
        assert st["grid"] <= grid
    assert_x_close(host(x), xo, what=f"rka q={q} grid={grid} mode={allreduce}")


def test_rka_two_phase_exchange_with_more_workgroups_than_threads():
    """2000 FP64 columns at q = 17: more workgroups than threads per workgroup,
    so a reducer polls some slots in a second round (under the bounded wait)."""
    say("rka G > NT")
    A, _, b = _system(3000, 2000, seed=17)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=17, max_iter=30, seed=9,
                               steps_per_exchange=1)
    assert info.status == rka.OK and st["kernel"] == 1 and st["variant"] == 0
    assert st["grid"] > st["threads"], st
    xo, _ = oracle.rka(A, b, q=17, max_iter=30, seed=9)
    assert_x_close(host(x), xo, what="rka G > NT")


def test_rka_small_q_on_rows_too_long_for_the_small_grid():
    """120000 FP64 columns at q = 8: slices of 120000 / 48 columns do not fit a
    workgroup, so the one-iteration kernel takes a wider grid (no fallback to
    the worker kernel, whose iterate would not fit)."""
    say("rka long rows q=8")
    A, _, b = _system(600, 120000, seed=19)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=8, max_iter=6, seed=5,
                               steps_per_exchange=1)
    assert info.status == rka.OK and st["kernel"] == 1 and st["grid"] > 48, st
    xo, _ = oracle.rka(A, b, q=8, max_iter=6, seed=5)
    assert_x_close(host(x), xo, what="rka long rows")


def test_rka_wide_q_falls_back_to_worker_kernel():
    # q rows per slice beyond the column kernel's tile: same iteration, other kernel
    say("rka q=2000")
    A, _, b = _system(3000, 64, seed=3)
    x, info = rka.rka_solve(to_dev(A), vec(b), q=2000, max_iter=5, seed=2)
    xo, _ = oracle.rka(A, b, q=2000, max_iter=5, seed=2)
    assert_x_close(host(x), xo, what="rka q=2000")


# -- stopping rule, determinism, resume, errors --------------------------------

def _oracle_measure(A, b, x, xs):
    """The stopping measure of a solve on x: error to xs, else the relative
    residual."""
    if xs is not None:
        return np.linalg.norm(x - xs) / np.linalg.norm(xs)
    return np.linalg.norm(b - A @ x) / np.linalg.norm(b)


def _same_stop(info, io, A, b, x_oracle_at, xs, tol, ce):
    """The GPU stops at the oracle's iteration; a different count is accepted
    only where the two sides' measures sit within rounding of tol at the
    earlier of the two test points (a tie the summation order decides)."""
    if info.iterations == io["iterations"]:
        return
    k = min(info.iterations, io["iterations"])
    meas = _oracle_measure(A, b, x_oracle_at(k), xs)
    assert abs(info.iterations - io["iterations"]) == ce and abs(meas - tol) <= 1e-12 * tol, (
        info.iterations, io["iterations"], meas)


@pytest.mark.parametrize("block", [0, 1, 5])
def test_stop_on_reference_error(block):
    say(f"stop x_ref block={block}")
    A, xs, b = workloads.gaussian_system(4000, 200, seed=workloads.DATA_SEED)
    Ad, bd, xd = to_dev(A), vec(b), vec(xs)
    if block == 0:
        x, info = rka.rka_solve(Ad, bd, q=8, max_iter=200000, tol=1e-8, seed=1, x_ref=xd)
        xo, io = oracle.rka(A, b, q=8, max_iter=200000, tol=1e-8, seed=1, x_ref=xs)

        def at(k):
            return oracle.rka(A, b, q=8, max_iter=k, seed=1)[0]
    else:
        x, info = rka.rkab_solve(Ad, bd, q=8, block_size=block, max_iter=200000, tol=1e-8,
                                 seed=1, x_ref=xd)
        xo, io = oracle.rkab(A, b, q=8, block_size=block, max_iter=200000, tol=1e-8, seed=1,
                             x_ref=xs)

        def at(k):
            return oracle.rkab(A, b, q=8, block_size=block, max_iter=k, seed=1)[0]
    assert info.status == rka.OK and io["status"] == oracle.OK
    _same_stop(info, io, A, b, at, xs, 1e-8, 1)
    assert np.linalg.norm(host(x) - xs) <= 1e-8 * np.linalg.norm(xs)
    # the stopped iterate against the oracle's iterate after the same count
    assert_x_close(host(x), at(info.iterations), what="stopped iterate")


def test_stop_on_residual():
    say("stop residual")
    A, xs, b = workloads.gaussian_system(1200, 60, seed=4)
    x, info = rka.rka_solve(to_dev(A), vec(b), q=4, max_iter=100000, tol=1e-7, seed=3,
                            check_every=25)
    xo, io = oracle.rka(A, b, q=4, max_iter=100000, tol=1e-7, seed=3, check_every=25)
    assert info.status == rka.OK and info.iterations % 25 == 0

    def at(k):
        return oracle.rka(A, b, q=4, max_iter=k, seed=3)[0]
    _same_stop(info, io, A, b, at, None, 1e-7, 25)
    xh = host(x)
    assert np.linalg.norm(b - A @ xh) <= 1e-7 * np.linalg.norm(b)
    assert_x_close(xh, at(info.iterations), what="stopped iterate (residual test)")


def test_not_converged_returns_last_iterate():
    A, xs, b = workloads.gaussian_system(500, 40, seed=6)
    x, info = rka.rka_solve(to_dev(A), vec(b), q=2, max_iter=30, tol=1e-12, seed=3,
                            x_ref=vec(xs))
    xo, io = oracle.rka(A, b, q=2, max_iter=30, tol=1e-12, seed=3, x_ref=xs)
    assert info.status == rka.NOT_CONVERGED == io["status"] and info.iterations == 30
    assert_x_close(host(x), xo)


@pytest.mark.parametrize("block", [0, 3])
def test_deterministic_and_resumable(block):
    say(f"determinism block={block}")
    A, _, b = _system(2000, 1000, seed=8)
    Ad, bd = to_dev(A), vec(b)

    def run(K, x0=None, off=0):
        if block == 0:
            return host(rka.rka_solve(Ad, bd, q=16, max_iter=K, seed=4, x0=x0, iter_offset=off)[0])
        return host(rka.rkab_solve(Ad, bd, q=16, block_size=block, max_iter=K, seed=4, x0=x0,
                                   iter_offset=off)[0])

    # bitwise across a split that falls on a block boundary (RKA at q = 16
    # runs blocks of 8 iterations per exchange by default)
    full = run(32)
    assert np.array_equal(full, run(32))
    half = run(16)
    rest = run(16, x0=vec(half), off=16)
    assert np.array_equal(full, rest)


def test_errors_reported():
    say("errors")
    A = np.zeros((40, 8))
    with pytest.raises(rka.RKAError) as e:
        rka.rka_solve(to_dev(A), vec(np.ones(40)), q=2, max_iter=3)
    assert e.value.status == rka.EZERONORM
    A, _, b = _system(40, 8)
    b[5] = np.nan
    with pytest.raises(rka.RKAError) as e:
        rka.rkab_solve(to_dev(A), vec(b), q=2, block_size=2, max_iter=3)
    assert e.value.status == rka.EINVAL
    with pytest.raises(rka.RKAError) as e:
        rka.rka_solve(to_dev(A), vec(np.ones(40)), q=0, max_iter=3)
    assert e.value.status == rka.EINVAL
    # large relaxation with duplicated rows: reported as diverged, not a crash
    A, _, b = _system(40, 8, noise=0)
    Ad = np.vstack([A, A])
    bd = np.concatenate([b, b + 1.0])
    _, info = rka.rka_solve(to_dev(Ad), vec(bd), q=1, alpha=50.0, max_iter=2000, tol=1e-12,
                            seed=1, check_every=50, raise_on_error=False)
    assert info.status == rka.EDIVERGED
