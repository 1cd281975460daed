"""GPU parity of RKA with several iterations per exchange, with the row inner
products formed inside the exchange (kernel 3, rka_block = 1; the block form
of Eq. (7) whose later dot products come from the first through the row inner
products): FP64 x within 1e-12 of the oracle on the same row stream for
block lengths 2..8, ragged q, ragged chunks and offsets, the scalar and
vector paths and narrow storage; the stopping test at the same iteration as
the one-iteration kernel; cyclic order and row weights; determinism; the
fallback when the block does not fit."""
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


CASES = [  # m, n, q, p, K, offset, dtype
    (3000, 2000, 16, 4, 40, 0, "f64"),
    (3000, 2000, 16, 2, 41, 7, "f64"),    # K not a multiple of p, offset
    (3000, 2000, 16, 3, 30, 0, "f64"),
    (2000, 1500, 8, 8, 33, 0, "f64"),
    (2000, 1500, 32, 2, 21, 3, "f64"),
    (1500, 777, 5, 3, 25, 0, "f64"),      # q not a multiple of 4, scalar path (odd n)
    (1500, 4096, 12, 5, 23, 0, "f64"),
    (5000, 10000, 16, 4, 16, 0, "f64"),   # slices of 40 columns
    (2000, 3000, 16, 4, 20, 0, "f32"),    # narrow storage, FP64 arithmetic
    (2000, 3000, 16, 4, 20, 0, "bf16"),
]


@pytest.mark.parametrize("m,n,q,p,K,off,dtype", CASES)
def test_sstep_vs_oracle(m, n, q, p, K, off, dtype):
    say(f"sstep {dtype} m={m} n={n} q={q} p={p} K={K} off={off}")
    A, _, b = workloads.gaussian_system(m, n, seed=31, noise_var=1e-2, dtype=dtype)
    A = np.array(A)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=0, q=q, alpha=1.1, max_iter=K,
                               seed=6, iter_offset=off, steps_per_exchange=p,
                               rka_block=1)
    assert info.status == rka.OK and info.iterations == K
    assert st["kernel"] == 3 and st["variant"] == p
    odt = "bf16" if dtype == "bf16" else None
    idx = oracle.indices(oracle.row_norms(A, dtype=odt), 6, off, K, q)
    xo = oracle.rka_given(A, b, np.zeros(n), idx, q=q, alpha=1.1, dtype=odt)
    assert_x_close(host(x), xo, 1e-12, "sstep")


@pytest.mark.parametrize("check_every,p", [(10, 4), (6, 4), (7, 3)])
def test_sstep_stops_where_the_one_iteration_kernel_stops(check_every, p):
    A, xs, b = workloads.gaussian_system(4000, 200, seed=32)
    A = np.array(A)
    kw = dict(method=0, q=16, alpha=8.0, max_iter=20000, tol=1e-8, x_ref=vec(xs),
              check_every=check_every, seed=2)
    x1, i1, s1 = rka.solve_ex(to_dev(A), vec(b), steps_per_exchange=1, **kw)
    xp, ip, sp = rka.solve_ex(to_dev(A), vec(b), steps_per_exchange=p, rka_block=1, **kw)
    assert s1["kernel"] == 1 and sp["kernel"] == 3
    assert i1.status == rka.OK and ip.status == rka.OK
    assert ip.iterations == i1.iterations and ip.iterations % check_every == 0
    assert_x_close(host(xp), host(x1), 1e-12, "stop")


def test_sstep_cyclic_order_and_row_weights():
    A, _, b = workloads.paper_rows_system(1800, 1200, seed=33)
    wrow = np.random.default_rng(33).uniform(0.5, 1.5, size=1800)
    K = 30
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=16, max_iter=K, sampling=2,
                               row_weight=vec(wrow), steps_per_exchange=4, rka_block=1)
    assert st["kernel"] == 3
    xo = oracle.rka_wrow_given(A, b, np.zeros(1200), oracle.indices_cyclic(1800, 0, K, 16, 1),
                               wrow, q=16)
    assert_x_close(host(x), xo, 1e-12, "cyclic sstep")


def test_sstep_is_deterministic():
    A, _, b = workloads.gaussian_system(3000, 2500, seed=34, noise_var=1e-2)
    Ad, bd = to_dev(np.array(A)), vec(b)
    xa, _, _ = rka.solve_ex(Ad, bd, method=0, q=16, max_iter=50, seed=3, steps_per_exchange=4,
                            rka_block=1)
    xb, _, _ = rka.solve_ex(Ad, bd, method=0, q=16, max_iter=50, seed=3, steps_per_exchange=4,
                            rka_block=1)
    assert np.array_equal(host(xa), host(xb))


def test_sstep_falls_back_when_the_block_does_not_fit():
    A, _, b = workloads.gaussian_system(2000, 1000, seed=35)
    A = np.array(A)
    # q p = 128 rows exceed the block tile: the one-iteration kernel runs
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=32, max_iter=10,
                               steps_per_exchange=4, rka_block=1)
    assert st["kernel"] == 1
    idx = oracle.indices(oracle.row_norms(A), 1, 0, 10, 32)
    assert_x_close(host(x), oracle.rka_given(A, b, np.zeros(1000), idx, q=32), 1e-12, "fallback")
    with pytest.raises(rka.RKAError) as e:
        rka.solve_ex(to_dev(A), vec(b), method=0, q=4, max_iter=3, steps_per_exchange=-1)
    assert e.value.status == rka.EINVAL


# -- RKAB split over columns (one outer iteration per exchange) -----------------

RKAB_CASES = [  # m, n, q, bs, K, dtype, sub-block length the library picks
    (3000, 2000, 16, 10, 12, "f64", 10),
    (2000, 1500, 8, 5, 20, "f64", 5),        # odd bs: unaligned tile reads
    (1500, 777, 6, 7, 15, "f64", 7),         # scalar path (odd n)
    (5000, 10000, 16, 10, 6, "f64", 10),     # 160 rows of 40-column slices: the 8-row tile
    (2000, 3000, 12, 4, 10, "f32", 4),       # narrow storage, FP64 arithmetic
    (2000, 3000, 12, 4, 10, "bf16", 4),
    (3000, 2000, 16, 40, 5, "f64", 16),      # sub-blocks 16, 16, 8
    (2000, 1200, 4, 150, 3, "f64", None),    # long blocks: ragged last sub-block
    (1500, 777, 6, 50, 4, "f64", None),      # sub-blocks on the scalar path
]


@pytest.mark.parametrize("m,n,q,bs,K,dtype,c", RKAB_CASES)
def test_rkab_column_split_vs_oracle(m, n, q, bs, K, dtype, c):
    say(f"rkab split {dtype} m={m} n={n} q={q} bs={bs} K={K}")
    A, _, b = workloads.gaussian_system(m, n, seed=36, noise_var=1e-2, dtype=dtype)
    A = np.array(A)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=1, q=q, block_size=bs,
                               alpha=0.9, max_iter=K, seed=7, rkab_split=2, rka_block=1)
    assert info.status == rka.OK and info.iterations == K and info.projections == K * q * bs
    assert st["kernel"] == 3 and 1 <= st["variant"] <= bs
    if c is not None:
        assert st["variant"] == c
    else:
        assert st["variant"] < bs  # sub-blocks
    odt = "bf16" if dtype == "bf16" else None
    idx = oracle.indices(oracle.row_norms(A, dtype=odt), 7, 0, K, q, bs)
    xo = oracle.rkab_given(A, b, np.zeros(n), idx, q=q, block_size=bs, alpha=0.9, dtype=odt)
    assert_x_close(host(x), xo, 1e-12, "rkab split")


def test_rkab_column_split_stops_where_the_worker_kernel_stops():
    A, xs, b = workloads.gaussian_system(4000, 300, seed=37)
    A = np.array(A)
    kw = dict(method=1, q=8, block_size=6, max_iter=20000, tol=1e-8, x_ref=vec(xs),
              check_every=5, seed=3)
    x1, i1, s1 = rka.solve_ex(to_dev(A), vec(b), rkab_split=1, **kw)
    x2, i2, s2 = rka.solve_ex(to_dev(A), vec(b), rkab_split=2, rka_block=1, **kw)
    assert s1["kernel"] == 2 and s2["kernel"] == 3
    assert i1.status == rka.OK and i2.status == rka.OK
    assert i2.iterations == i1.iterations and i2.iterations % 5 == 0
    assert_x_close(host(x2), host(x1), 1e-12, "rkab split stop")


def test_rkab_sub_blocks_stop_where_the_worker_kernel_stops():
    A, xs, b = workloads.gaussian_system(3000, 400, seed=40)
    A = np.array(A)
    kw = dict(method=1, q=4, block_size=90, max_iter=5000, tol=1e-9, x_ref=vec(xs),
              check_every=2, seed=5)
    x1, i1, s1 = rka.solve_ex(to_dev(A), vec(b), rkab_split=1, **kw)
    x2, i2, s2 = rka.solve_ex(to_dev(A), vec(b), rkab_split=2, rka_block=1, **kw)
    assert s1["kernel"] == 2 and s2["kernel"] == 3 and s2["variant"] < 90
    assert i1.status == rka.OK and i2.status == rka.OK
    assert i2.iterations == i1.iterations
    assert_x_close(host(x2), host(x1), 1e-12, "rkab sub-block stop")


def test_rkab_column_split_cyclic_and_row_weights():
    A, _, b = workloads.paper_rows_system(1500, 900, seed=38)
    wrow = np.random.default_rng(38).uniform(0.5, 1.5, size=1500)
    K, q, bs = 12, 10, 30  # sub-blocks of 25 and 5
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=1, q=q, block_size=bs, max_iter=K,
                               sampling=2, row_weight=vec(wrow), rkab_split=2, rka_block=1)
    assert st["kernel"] == 3
    xo = oracle.rkab_wrow_given(A, b, np.zeros(900), oracle.indices_cyclic(1500, 0, K, q, bs),
                                wrow, q=q, block_size=bs)
    assert_x_close(host(x), xo, 1e-12, "rkab split cyclic")


def test_rkab_column_split_falls_back_and_checks_arguments():
    A, _, b = workloads.gaussian_system(2000, 500, seed=39)
    A = np.array(A)
    # more than 256 workers: not even one row per worker fits the block tile
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=1, q=300, block_size=2, max_iter=3,
                               seed=2, rkab_split=2)
    assert st["kernel"] == 2
    idx = oracle.indices(oracle.row_norms(A), 2, 0, 3, 300, 2)
    assert_x_close(host(x), oracle.rkab_given(A, b, np.zeros(500), idx, q=300, block_size=2),
                   1e-12, "rkab fallback")
    with pytest.raises(rka.RKAError) as e:
        rka.solve_ex(to_dev(A), vec(b), method=1, q=4, block_size=3, max_iter=3, rkab_split=3)
    assert e.value.status == rka.EINVAL
