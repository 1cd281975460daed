"""GPU parity of the cyclic row order (Sec. 2.1) and the per-row weights of
Eq. (7) through the C ABI, and of RKA on the coherent-row workload of
Sec. 3.1: FP64 iterates within 1e-12 of the oracle on the same row stream
(Cyclic Kaczmarz itself at q = 1), FP32 accumulation within its rounding
bound, zero rows as no-op steps, argument errors."""
import numpy as np
import pytest

import oracle
import workloads
from bars import binary32_bar, oracle_pair, rel
from gpu_util import assert_x_close, host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


@pytest.mark.parametrize("m,n,iters", [(700, 64, 3000), (300, 2500, 700), (50, 9000, 120)])
def test_cyclic_kaczmarz_vs_oracle(m, n, iters):
    say(f"ck m={m} n={n} iters={iters}")
    A, _, b = workloads.paper_rows_system(m, n, seed=21)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=1, max_iter=iters, sampling=2)
    assert info.status == rka.OK and info.projections == iters
    assert_x_close(host(x), oracle.ck(A, b, iters=iters), 1e-12, "ck")


CASES = [  # m, n, q, bs, K, offset, grid
    (1000, 128, 8, 1, 200, 0, 0),
    (777, 3000, 16, 1, 40, 13, 0),     # many workgroups, ragged wrap of the rows
    (777, 3000, 16, 1, 40, 13, 12),    # one-barrier all-gather
    (900, 200, 64, 1, 30, 5, 0),
    (500, 300, 4, 7, 20, 3, 0),        # RKAB
    (400, 9000, 3, 5, 6, 0, 0),        # RKAB, iterate in LDS
]


@pytest.mark.parametrize("m,n,q,bs,K,off,grid", CASES)
def test_cyclic_stream_vs_oracle(m, n, q, bs, K, off, grid):
    say(f"cyclic m={m} n={n} q={q} bs={bs} K={K} off={off} grid={grid}")
    A, _, b = workloads.gaussian_system(m, n, seed=22, noise_var=1e-2)
    A = np.array(A)
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=0 if bs == 1 else 1, q=q,
                              block_size=bs, alpha=1.2, max_iter=K, seed=1, iter_offset=off,
                              grid=grid, sampling=2)
    assert info.status == rka.OK
    idx = oracle.indices_cyclic(m, off, K, q, bs)
    if bs == 1:
        xo = oracle.rka_given(A, b, np.zeros(n), idx, q=q, alpha=1.2)
    else:
        xo = oracle.rkab_given(A, b, np.zeros(n), idx, q=q, block_size=bs, alpha=1.2)
    assert_x_close(host(x), xo, 1e-12, "cyclic")


@pytest.mark.parametrize("m,n,q,bs,K", [(1500, 96, 8, 1, 80), (1200, 2500, 16, 1, 30),
                                        (800, 400, 6, 4, 15)])
def test_row_weights_vs_oracle(m, n, q, bs, K):
    say(f"row weights m={m} n={n} q={q} bs={bs} K={K}")
    A, _, b = workloads.scaled_rows_system(m, n, seed=23, noise_var=1e-2)
    A = np.array(A)
    wrow = np.random.default_rng(23).uniform(0.3, 1.7, size=m)
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=0 if bs == 1 else 1, q=q,
                              block_size=bs, max_iter=K, seed=8, row_weight=vec(wrow))
    assert info.status == rka.OK
    idx = oracle.indices(oracle.row_norms(A), 8, 0, K, q, bs)
    if bs == 1:
        xo = oracle.rka_wrow_given(A, b, np.zeros(n), idx, wrow, q=q)
    else:
        xo = oracle.rkab_wrow_given(A, b, np.zeros(n), idx, wrow, q=q, block_size=bs)
    assert_x_close(host(x), xo, 1e-12, "row weights")


@pytest.mark.parametrize("method,bs", [(0, 1), (1, 3)])
def test_cyclic_zero_rows_are_no_ops(method, bs):
    A, _, b = workloads.gaussian_system(300, 80, seed=24)
    A = np.array(A)
    A[[0, 17, 299]] = 0.0
    b = b.copy()
    b[17] = 5.0  # a zero row with b_i != 0 has no hyperplane: its step is skipped
    wrow = np.random.default_rng(24).uniform(0.5, 1.5, size=300)
    K = 40
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=method, q=5, block_size=bs, max_iter=K,
                              sampling=2, row_weight=vec(wrow))
    assert info.status == rka.OK
    idx = oracle.indices_cyclic(300, 0, K, 5, bs)
    if bs == 1:
        xo = oracle.rka_wrow_given(A, b, np.zeros(80), idx, wrow, q=5)
    else:
        xo = oracle.rkab_wrow_given(A, b, np.zeros(80), idx, wrow, q=5, block_size=bs)
    xg = host(x)
    assert np.all(np.isfinite(xg))
    assert_x_close(xg, xo, 1e-12, "zero rows")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_cyclic_fp32_accumulation_vs_oracle(dtype):
    m, n, q, K = 900, 2048, 8, 25
    A, _, b = workloads.gaussian_system(m, n, seed=25, noise_var=1e-2, dtype=dtype)
    A = np.array(A)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=0, q=q, max_iter=K,
                               accumulate=1, sampling=2)
    assert info.status == rka.OK and st["accumulate"] == 1
    odt = "bf16" if dtype == "bf16" else None
    xo, x64 = oracle_pair(oracle, A, b, np.zeros(n), oracle.indices_cyclic(m, 0, K, q, 1), q=q,
                          dtype=odt)
    gap, bar = rel(host(x), xo), binary32_bar(xo, x64)
    assert gap <= bar, (gap, bar)


@pytest.mark.parametrize("m,n,q", [(4000, 200, 16), (2000, 3000, 64)])
def test_coherent_rows_workload_vs_oracle(m, n, q):
    say(f"coherent rows m={m} n={n} q={q}")
    A, _, b = workloads.paper_rows_system(m, n, seed=26)
    K = 30
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=0, q=q, max_iter=K, seed=12)
    assert info.status == rka.OK
    idx = oracle.indices(oracle.row_norms(A), 12, 0, K, q)
    assert_x_close(host(x), oracle.rka_given(A, b, np.zeros(n), idx, q=q), 1e-12, "coherent")


def test_sampling_and_weight_arguments():
    A, _, b = workloads.gaussian_system(60, 8, seed=27)
    A = np.array(A)
    for bad in (-1, 3):
        with pytest.raises(rka.RKAError) as e:
            rka.solve_ex(to_dev(A), vec(b), method=0, q=2, max_iter=3, sampling=bad)
        assert e.value.status == rka.EINVAL
    with pytest.raises(rka.RKAError) as e:
        rka.solve_ex(to_dev(A), vec(b), method=0, q=2, max_iter=3, worker_alpha=vec(np.ones(2)),
                     row_weight=vec(np.ones(60)))
    assert e.value.status == rka.EINVAL
