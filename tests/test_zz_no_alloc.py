"""rka_solve_ex_noalloc, the allocation-free variant of rka_solve_ex (scratch
from the library's fixed device array), against rka_solve_ex through the C
ABI: two calls in a row on each kernel, the second with a smaller input, and
the rejection of a problem whose buffers exceed the array.

Bar: the same iteration count and status, and x bitwise equal to
rka_solve_ex's where the row records of a chunk fit the array (the same
chunks, so the same arithmetic), else within 1e-12 in FP64 (shorter chunks
move the block ends of RKA with several iterations per exchange).
"""
import numpy as np
import pytest

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


def _run(A, b, no_alloc, **kw):
    x, info, st = rka.solve_ex(A, b, no_alloc=no_alloc, raise_on_error=False, **kw)
    torch.cuda.synchronize()
    return x, info, st


PAIRS = [
    # (first call, second call with a smaller input): kernel each reaches
    ((0, 2500, 1000, 16, 1, 40), (0, 900, 200, 16, 1, 30)),    # several iterations per exchange
    ((0, 3000, 1024, 64, 1, 25), (0, 2000, 96, 8, 1, 50)),     # column-split RKA
    ((1, 2000, 1000, 16, 10, 8), (1, 700, 48, 8, 4, 20)),      # column-split RKAB
    ((1, 3000, 513, 300, 2, 4), (1, 600, 77, 40, 3, 6)),       # worker-split RKAB
]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_matches_solve_ex_twice(first, second):
    for (method, m, n, q, bs, K) in (first, second):
        say(f"noalloc method={method} {m}x{n} q={q} bs={bs} K={K}")
        A, xs, b = workloads.gaussian_system(m, n, seed=m + n, noise_var=0.01)
        Ad, bd = to_dev(A), vec(b)
        kw = dict(method=method, q=q, block_size=bs, alpha=1.0, max_iter=K, seed=5)
        x0, i0, s0 = _run(Ad, bd, False, **kw)
        x1, i1, s1 = _run(Ad, bd, True, **kw)
        assert i0.status == i1.status == rka.OK and i0.iterations == i1.iterations == K
        assert s1["kernel"] == s0["kernel"] and s1["iterate_launches"] == s0["iterate_launches"]
        assert torch.equal(x0, x1)


def test_noalloc_stops_like_solve_ex():
    """A residual-measured stop (which uses the partial-sum buffer) and an
    x_ref stop, in a row on the same device array."""
    say("noalloc stopping")
    A, xs, _ = workloads.gaussian_system(4000, 200, seed=5)
    b = A @ xs
    Ad, bd = to_dev(A), vec(b)
    for kw in (dict(tol=1e-8, x_ref=vec(xs), check_every=1),
               dict(tol=1e-6, check_every=50)):
        x0, i0, _ = _run(Ad, bd, False, method=0, q=8, max_iter=200000, seed=3, **kw)
        x1, i1, _ = _run(Ad, bd, True, method=0, q=8, max_iter=200000, seed=3, **kw)
        assert i0.status == i1.status == rka.OK and i0.iterations == i1.iterations
        assert torch.equal(x0, x1)


def test_noalloc_shorter_chunks_within_bar():
    """Row records of 2.56 M projections (82 MB) exceed the array: the
    allocation-free call runs more, shorter chunks; same iteration count,
    x within 1e-12."""
    say("noalloc chunked")
    A, _, b = workloads.gaussian_system(3000, 256, seed=2, noise_var=0.01)
    Ad, bd = to_dev(A), vec(b)
    kw = dict(method=0, q=256, max_iter=10000, seed=7)
    x0, i0, s0 = _run(Ad, bd, False, **kw)
    x1, i1, s1 = _run(Ad, bd, True, **kw)
    assert i0.status == i1.status == rka.OK and i0.iterations == i1.iterations == 10000
    assert s1["iterate_launches"] > s0["iterate_launches"]
    assert_x_close(host(x1), host(x0), what="noalloc chunked")
    # and a smaller problem right after, on the same array
    A2, _, b2 = workloads.gaussian_system(500, 40, seed=3, noise_var=0.01)
    x2, i2, _ = _run(to_dev(A2), vec(b2), True, method=1, q=4, block_size=3, max_iter=9, seed=1)
    x3, i3, _ = _run(to_dev(A2), vec(b2), False, method=1, q=4, block_size=3, max_iter=9, seed=1)
    assert i2.status == i3.status == rka.OK and torch.equal(x2, x3)


def test_noalloc_rejects_problems_beyond_the_array():
    """5e6 rows need 80 MB of norms and running sums: RKA_EINVAL before any
    launch, with a message naming the limit; the allocating call still runs."""
    say("noalloc too large")
    m = 5_000_000
    A = torch.ones((m, 1), dtype=torch.float64, device="cuda:0")
    b = torch.ones(m, dtype=torch.float64, device="cuda:0")
    x, info, _ = _run(A, b, True, method=0, q=4, max_iter=3, seed=1)
    assert info.status == rka.EINVAL
    msg = rka.lib().rka_last_error().decode()
    assert "allocation-free scratch" in msg and str(64 << 20) in msg
    x, info, _ = _run(A, b, False, method=0, q=4, max_iter=3, seed=1)
    assert info.status == rka.OK
    assert np.allclose(host(x), 1.0)
