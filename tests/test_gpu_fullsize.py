"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (library defaults): the 80000 x 10000 FP64 system with
b = A x* + N(0, 1e-2), and the 200000 x 20000 BF16 system of the precision
form.  The oracle's cost per iteration is q bs n (independent of m), so it runs
a few iterations of every cell of the benchmark grid at full size on the same
row stream: row norms and the stream bit-exact, FP64 x within 1e-12, the FP32
inner iteration within its rounding bound."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_x_close, host, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def main_system():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()
    say("full size: generating 80000 x 10000 FP64")
    A, _, b = workloads.gaussian_system(80000, 10000, seed=workloads.DATA_SEED, noise_var=1e-2,
                                        rng="torch", device=torch.device("cuda:0"))
    Ah = A.cpu().numpy()
    bh = b.cpu().numpy()
    say("full size: oracle row norms")
    w = oracle.row_norms(Ah)
    yield A, b, Ah, bh, w
    del A, b
    torch.cuda.empty_cache()


def test_fullsize_norms_and_stream_bitwise(main_system):
    A, b, Ah, bh, w = main_system
    wg = rka.row_norms(A)
    assert np.array_equal(host(wg), w)
    c, _ = rka.prefix(wg)
    idx = host(rka.sample_indices(wg, c, seed=11, iter_offset=123456, K=40, q=256, bs=1))
    assert np.array_equal(idx, oracle.indices(w, 11, 123456, 40, 256, 1))


# the benchmark's cells (method, q, block size), a few iterations each
CELLS = [("rka", 16, 1, 40), ("rka", 64, 1, 16), ("rka", 256, 1, 6), ("rkab", 16, 10, 4),
         ("rkab", 16, 100, 2), ("rkab", 64, 10, 3), ("rkab", 256, 100, 1)]


@pytest.mark.parametrize("meth,q,bs,K", CELLS)
def test_fullsize_cells_vs_oracle(main_system, meth, q, bs, K):
    A, b, Ah, bh, w = main_system
    say(f"full size {meth} q={q} bs={bs} K={K}")
    alpha = 1.0 if meth == "rkab" else 1.3
    x, info, st = rka.solve_ex(A, b, method=0 if meth == "rka" else 1, q=q, block_size=bs,
                               alpha=alpha, max_iter=K, seed=17)
    assert info.status == rka.OK and info.projections == K * q * bs
    idx = oracle.indices(w, 17, 0, K, q, bs)
    if meth == "rka":
        xo = oracle.rka_given(Ah, bh, np.zeros(10000), idx, q=q, alpha=alpha)
    else:
        xo = oracle.rkab_given(Ah, bh, np.zeros(10000), idx, q=q, block_size=bs, alpha=alpha)
    assert_x_close(host(x), xo, 1e-12, f"full size {meth} q={q} bs={bs} (kernel {st['kernel']})")


def test_fullsize_precision_inner_vs_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()
    say("full size: generating 200000 x 20000 BF16")
    A, _, b = workloads.gaussian_system(200000, 20000, seed=workloads.DATA_SEED + 2,
                                        noise_var=1e-4, dtype="bf16", rng="torch",
                                        device=torch.device("cuda:0"))
    Ah = A.view(torch.int16).cpu().numpy().view(np.uint16)
    bh = b.cpu().numpy()
    q, K = 64, 4
    x, info, st = rka.solve_ex(A, b, method=0, q=q, max_iter=K, seed=19, accumulate=1)
    assert info.status == rka.OK and st["accumulate"] == 1
    say("full size: oracle FP32 iteration")
    w = oracle.row_norms(Ah, dtype="bf16")
    xo = oracle.rka_f32_given(Ah, bh, np.zeros(20000), oracle.indices(w, 19, 0, K, q), q=q,
                              dtype="bf16")
    del A, b
    torch.cuda.empty_cache()
    gap = np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)
    assert gap <= 4 * K * 20000 * U32, gap
