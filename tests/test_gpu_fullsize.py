"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times (library defaults, solves through a plan of A): the
80000 x 10000 FP64 system with b = A x* + N(0, 1e-2), and the 200000 x 20000
system of the precision form stored as BF16 and as FP32.  The oracle's cost
per iteration is q bs n (independent of m), so it runs a few iterations of
every cell of the benchmark grid at full size on the same row stream: row
norms and the stream bit-exact, FP64 x within 1e-12, the FP32-arithmetic
inner iteration and one refinement sweep within the binary32 bar of
tests/bars.py."""
import numpy as np
import pytest

import oracle
import workloads
from bars import binary32_bar, oracle_pair, rel
from gpu_util import assert_x_close, host, say, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

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
    P = rka.Plan(A)
    yield A, b, Ah, bh, w, P
    P.close()
    del A, b
    torch.cuda.empty_cache()


def test_fullsize_norms_and_stream_bitwise(main_system):
    A, b, Ah, bh, w, P = main_system
    wg = rka.row_norms(A)
    assert np.array_equal(host(wg), w)
    assert np.array_equal(host(P.row_norms()), w)
    c, _ = rka.prefix(wg)
    idx = host(rka.sample_indices(wg, c, seed=11, iter_offset=123456, K=40, q=256, bs=1))
    assert np.array_equal(idx, oracle.indices(w, 11, 123456, 40, 256, 1))
    idx = host(P.sample_indices(seed=12, iter_offset=99, K=30, q=64, bs=10))
    assert np.array_equal(idx, oracle.indices(w, 12, 99, 30, 64, 10))


# every cell of the benchmark grid (method, q, block size), a few iterations each
CELLS = [("rka", 16, 1, 40), ("rka", 64, 1, 16), ("rka", 256, 1, 6), ("rkab", 16, 10, 4),
         ("rkab", 16, 100, 2), ("rkab", 64, 10, 3), ("rkab", 64, 100, 1), ("rkab", 256, 10, 2),
         ("rkab", 256, 100, 1)]


@pytest.mark.parametrize("meth,q,bs,K", CELLS)
def test_fullsize_cells_vs_oracle(main_system, meth, q, bs, K):
    A, b, Ah, bh, w, P = main_system
    say(f"full size {meth} q={q} bs={bs} K={K}")
    alpha = 1.0 if meth == "rkab" else 1.3
    x, info, st = P.solve(b, method=0 if meth == "rka" else 1, q=q, block_size=bs,
                          alpha=alpha, max_iter=K, seed=17)
    assert info.status == rka.OK and info.projections == K * q * bs
    idx = oracle.indices(w, 17, 0, K, q, bs)
    if meth == "rka":
        xo = oracle.rka_given(Ah, bh, np.zeros(10000), idx, q=q, alpha=alpha)
    else:
        xo = oracle.rkab_given(Ah, bh, np.zeros(10000), idx, q=q, block_size=bs, alpha=alpha)
    assert_x_close(host(x), xo, 1e-12, f"full size {meth} q={q} bs={bs} (kernel {st['kernel']})")


@pytest.fixture(scope="module", params=["bf16", "f32"])
def precision_system(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()
    dt = request.param
    say(f"full size: generating 200000 x 20000 {dt}, b = A x* (consistent)")
    A, xs, b = workloads.gaussian_system(200000, 20000, seed=workloads.DATA_SEED + 2,
                                         noise_var=0.0, dtype=dt, rng="torch",
                                         device=torch.device("cuda:0"))
    del xs
    if dt == "bf16":
        Ah = A.view(torch.int16).cpu().numpy().view(np.uint16)
    else:
        Ah = A.cpu().numpy()
    bh = b.cpu().numpy()
    od = "bf16" if dt == "bf16" else None
    say("full size: oracle row norms")
    w = oracle.row_norms(Ah, dtype=od)
    yield dt, od, A, b, Ah, bh, w
    del A, b
    torch.cuda.empty_cache()


@pytest.mark.timeout(300)
def test_fullsize_precision_inner_vs_oracle(precision_system):
    """50 iterations of the FP32-arithmetic inner RKA (q = 64) at 200000 x 20000."""
    dt, od, A, b, Ah, bh, w = precision_system
    q, K = 64, 50
    say(f"full size {dt} inner RKA q={q} K={K}")
    x, info, st = rka.solve_ex(A, b, method=0, q=q, max_iter=K, seed=19, accumulate=1)
    assert info.status == rka.OK and st["accumulate"] == 1
    xo, x64 = oracle_pair(oracle, Ah, bh, np.zeros(20000), oracle.indices(w, 19, 0, K, q), q=q,
                          dtype=od)
    gap, bar = rel(host(x), xo), binary32_bar(xo, x64)
    say(f"  gap {gap:.3e}  bar {bar:.3e}")
    assert gap <= bar, (gap, bar)


@pytest.mark.timeout(300)
def test_fullsize_refinement_sweep_vs_oracle(precision_system):
    """One refinement sweep (FP64 residual over the whole matrix, binary32
    inner RKA q = 64 for 100 iterations, x += d) against the oracle's sweep on
    the same streams: within the binary32 bar of the oracle's binary32 and
    binary64 sweeps; the sweep measure likewise."""
    dt, od, A, b, Ah, bh, w = precision_system
    say(f"full size {dt} refinement sweep")
    x, ri = rka.refine_solve(A, b, method=0, q=64, accumulate=1, inner_iters=100, max_sweeps=1,
                             seed=23)
    assert ri.status == rka.OK and ri.sweeps == 1
    kw = dict(method=0, q=64, alpha=1.0, inner_iters=100, sweeps=1, seed=23, dtype=od)
    x32, m32 = oracle.refine(Ah, bh, acc32=1, **kw)
    x64, m64 = oracle.refine(Ah, bh, acc32=0, **kw)
    gap, bar = rel(host(x), x32), binary32_bar(x32, x64)
    say(f"  gap {gap:.3e}  bar {bar:.3e}")
    assert gap <= bar, (gap, bar)
    # |measure difference| <= ||A (x - x32)|| / ||A x*|| <= cond(A) gap ||x32|| / ||x*||,
    # with cond(A) < 2 for this iid Gaussian shape
    assert abs(ri.measures[0] - m32[0]) <= 4 * bar
