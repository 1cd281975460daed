"""Degenerate and edge cases through the C ABI: zero iterations, one row, one
column, more workers than rows, kernels asked for on shapes they cannot take,
and the minimum-norm limit of Sec. 2.1 on an underdetermined system."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_x_close, host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


@pytest.mark.parametrize("method,bs,split", [(0, 1, 0), (1, 3, 1), (1, 3, 2)])
def test_zero_iterations_return_the_start(method, bs, split):
    A, _, b = workloads.gaussian_system(300, 40, seed=41)
    x0 = np.random.default_rng(41).standard_normal(40)
    x, info, _ = rka.solve_ex(to_dev(np.array(A)), vec(b), method=method, q=4, block_size=bs,
                              max_iter=0, x0=vec(x0), rkab_split=split)
    assert info.status == rka.OK and info.iterations == 0 and info.projections == 0
    assert np.array_equal(host(x), x0)
    x, info, _ = rka.solve_ex(to_dev(np.array(A)), vec(b), method=method, q=4, block_size=bs,
                              max_iter=0, rkab_split=split)
    assert np.array_equal(host(x), np.zeros(40))


SHAPES = [(1, 1), (1, 7), (9, 1), (5, 40), (2, 3)]


@pytest.mark.parametrize("m,n", SHAPES)
@pytest.mark.parametrize("method,q,bs", [(0, 3, 1), (0, 12, 1), (1, 2, 2), (1, 7, 3)])
def test_tiny_shapes_vs_oracle(m, n, method, q, bs):
    say(f"tiny m={m} n={n} method={method} q={q} bs={bs}")
    g = np.random.default_rng(m * 100 + n)
    A = g.standard_normal((m, n)) * g.uniform(0.5, 2.0, size=(m, 1))
    b = g.standard_normal(m)
    K = 25
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=method, q=q, block_size=bs, alpha=0.9,
                              max_iter=K, seed=5)
    assert info.status == rka.OK and info.projections == K * q * bs
    if method == 0:
        xo, _ = oracle.rka(A, b, q=q, alpha=0.9, max_iter=K, seed=5)
    else:
        xo, _ = oracle.rkab(A, b, q=q, block_size=bs, alpha=0.9, max_iter=K, seed=5)
    assert_x_close(host(x), xo, 1e-12, f"tiny {m}x{n}")


def test_kernels_asked_for_on_shapes_they_cannot_take():
    b = np.random.default_rng(43).standard_normal(50)
    # three columns: the block kernel on three one-column workgroups
    A = np.random.default_rng(42).standard_normal((50, 3))
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=4, max_iter=12, seed=2,
                               steps_per_exchange=4, rka_block=1)
    assert st["kernel"] == 3 and st["grid"] == 3
    xo, _ = oracle.rka(A, b, q=4, max_iter=12, seed=2)
    assert_x_close(host(x), xo, 1e-12, "block kernel, one column per workgroup")
    # one column: a single slice has no exchange to save, the one-iteration kernel runs
    A1 = A[:, :1].copy()
    x, info, st = rka.solve_ex(to_dev(A1), vec(b), method=0, q=4, max_iter=12, seed=2,
                               steps_per_exchange=4)
    assert st["kernel"] == 1
    xo, _ = oracle.rka(A1, b, q=4, max_iter=12, seed=2)
    assert_x_close(host(x), xo, 1e-12, "block kernel fallback")
    # FP32 accumulation: the column split is FP64 only, the worker kernel runs
    A32 = A.astype(np.float32)
    x, info, st = rka.solve_ex(to_dev(A32), vec(b), method=1, q=2, block_size=3, max_iter=5,
                               seed=2, accumulate=1, rkab_split=2)
    assert st["kernel"] == 2 and st["accumulate"] == 1


@pytest.mark.parametrize("q", [1, 8])
def test_underdetermined_reaches_the_min_norm_solution(q):
    # Sec. 2.1: from x = 0, Kaczmarz on a consistent underdetermined system
    # converges to its minimum-norm solution
    g = np.random.default_rng(44)
    A = g.standard_normal((30, 200))
    b = g.standard_normal(30)
    want = np.linalg.pinv(A) @ b
    x, info = rka.rka_solve(to_dev(A), vec(b), q=q, max_iter=40000 // q, seed=3)
    assert info.status == rka.OK
    assert np.linalg.norm(host(x) - want) <= 1e-10 * np.linalg.norm(want)
