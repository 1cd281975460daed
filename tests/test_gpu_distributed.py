"""GPU parity of the Distributed Approach and the partial-matrix weights
(Sec. 3.3.2) through the C ABI: the block row stream bit-exact against the
oracle; RKA and RKAB with block sampling and/or per-worker weights within
1e-12 of the oracle on the same stream; per-worker weights from the device
Lanczos against numpy's SVD of every block."""
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


@pytest.mark.parametrize("m,q,bs,K", [(1, 1, 1, 5), (103, 7, 3, 40), (5000, 16, 2, 30),
                                      (80001, 256, 1, 4), (999, 999, 1, 2)])
def test_block_stream_bitwise(m, q, bs, K):
    say(f"sample_blocks m={m} q={q} bs={bs}")
    A, _, _ = workloads.scaled_rows_system(m, 16, seed=3)
    A = np.array(A)
    w = oracle.row_norms(A)
    idx = host(rka.sample_blocks(vec(w), seed=11, iter_offset=7, K=K, q=q, bs=bs))
    assert np.array_equal(idx, oracle.indices_blocks(w, 11, 7, K, q, bs))


CASES = [  # m, n, q, bs, K, grid, weights
    (1200, 64, 8, 1, 60, 0, False),
    (3000, 2000, 16, 1, 30, 0, True),
    (3000, 2000, 16, 1, 30, 12, True),   # one-barrier all-gather
    (2500, 1000, 64, 1, 20, 0, False),
    (1500, 300, 6, 5, 12, 0, True),      # RKAB
    (1500, 9000, 4, 3, 6, 0, True),      # RKAB, iterate in LDS
]


@pytest.mark.parametrize("m,n,q,bs,K,grid,weights", CASES)
def test_distributed_solve_vs_oracle(m, n, q, bs, K, grid, weights):
    say(f"distributed m={m} n={n} q={q} bs={bs} K={K} grid={grid} weights={weights}")
    A, _, b = workloads.gaussian_system(m, n, seed=5, noise_var=1e-2)
    A = np.array(A)
    wa = (np.linspace(0.6, 1.3, q) if weights else np.full(q, 0.8))
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0 if bs == 1 else 1, q=q,
                               block_size=bs, alpha=0.8, max_iter=K, seed=9, grid=grid,
                               sampling=1, worker_alpha=vec(wa) if weights else None)
    assert info.status == rka.OK
    idx = oracle.indices_blocks(oracle.row_norms(A), 9, 0, K, q, bs)
    if bs == 1:
        xo = oracle.rka_walpha_given(A, b, np.zeros(n), idx, wa, q=q)
    else:
        xo = oracle.rkab_walpha_given(A, b, np.zeros(n), idx, wa, q=q, block_size=bs)
    assert_x_close(host(x), xo, 1e-12, "distributed")


def test_worker_weights_with_full_matrix_sampling():
    A, _, b = workloads.gaussian_system(2000, 500, seed=6, noise_var=1e-2)
    A = np.array(A)
    q, K = 12, 40
    wa = np.linspace(0.5, 1.5, q)
    x, info, _ = rka.solve_ex(to_dev(A), vec(b), method=0, q=q, max_iter=K, seed=4,
                              worker_alpha=vec(wa))
    idx = oracle.indices(oracle.row_norms(A), 4, 0, K, q)
    assert_x_close(host(x), oracle.rka_walpha_given(A, b, np.zeros(500), idx, wa, q=q), 1e-12,
                   "weights")


@pytest.mark.parametrize("m,n,q", [(2000, 60, 4), (1200, 300, 8)])
def test_partial_alpha_vs_svd_of_each_block(m, n, q):
    A, _, _ = workloads.gaussian_system(m, n, seed=8)
    A = np.array(A)
    wa = host(rka.partial_alpha(to_dev(A), q, steps=min(m // q, n), seed=2))
    for w in range(q):
        blk = A[w * m // q:(w + 1) * m // q]
        sv = np.linalg.svd(blk, compute_uv=False)
        F = np.sum(sv ** 2)
        want = rka.alpha_star(sv[-1] ** 2 / F, sv[0] ** 2 / F, q)
        assert abs(wa[w] - want) <= 1e-8 * want, (w, wa[w], want)


def test_zero_weight_block_is_reported():
    A, _, b = workloads.gaussian_system(400, 10, seed=9)
    A = np.array(A)
    A[100:200] = 0.0  # the second of four blocks
    with pytest.raises(rka.RKAError) as e:
        rka.solve_ex(to_dev(A), vec(b), method=0, q=4, max_iter=5, sampling=1)
    assert e.value.status == rka.EZERONORM
