"""GPU parity of RKA in blocks of p iterations with coefficients from a
streaming pass (kernel 4, rka_block = 2): per block the scales are s = M c
with M = (I + N)^-1 formed ahead of the iterations from the inner products of
the block's rows (Eq. (7) unrolled over the block), and only the p q dot
products with x^(k) cross the chip.  The same iteration in exact arithmetic:
FP64 x within 1e-12 of the oracle on the same row stream, over block lengths,
ragged block and chunk ends, stopping tests, resumed streams, storage types,
row orders and weights, and launch geometries."""
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


def _system(m, n, dtype="f64", seed=1, noise=0.01):
    A, xs, b = workloads.gaussian_system(m, n, seed=seed, noise_var=noise, dtype=dtype)
    return np.array(A), xs, b


def _odt(dtype):
    return "bf16" if dtype == "bf16" else None


CASES = [
    # m, n, dtype, q, p (0: the library's), K, grid
    (3000, 2000, "f64", 16, 0, 40, 0),      # 8 iterations per block (the default), default grid
    (3000, 2000, "f64", 16, 8, 41, 0),      # 128 rows per block, ragged last block
    (3000, 2000, "f64", 8, 0, 37, 0),
    (3000, 2000, "f64", 4, 16, 50, 0),
    (3000, 2000, "f64", 32, 0, 20, 0),
    (3000, 2000, "f64", 64, 0, 15, 0),      # 2 iterations of 64 rows
    (3000, 2000, "f64", 5, 12, 33, 0),      # odd q, 60 rows
    (2500, 999, "f64", 16, 4, 30, 0),       # scalar path, ragged slice
    (2000, 1000, "f64", 16, 4, 30, 8),      # few workgroups, 64-lane row groups
    (2000, 1000, "f64", 16, 4, 30, 100),    # more workgroups than exchange values
    (1500, 4096, "f32", 16, 4, 30, 0),      # narrow storage, FP64 arithmetic
    (1500, 4096, "bf16", 12, 5, 30, 0),
    (700, 48, "f64", 8, 4, 25, 2),
    (3000, 2000, "f64", 256, 1, 6, 0),     # one iteration per block: no coefficients
    (3000, 2000, "f64", 128, 1, 8, 0),
    (5000, 10000, "f64", 16, 4, 24, 0),     # long rows: 24-vec (384-byte) slices, the last 8
    (3000, 7000, "f64", 16, 0, 40, 0),      # 16-vec slices (14 rounded up to a line), the last 12
    (1500, 20000, "f32", 16, 4, 24, 0),     # narrow storage, 24-vec slices
    (1000, 40000, "bf16", 16, 4, 16, 0),
]


@pytest.mark.parametrize("m,n,dtype,q,p,K,grid", CASES)
def test_blk_vs_oracle(m, n, dtype, q, p, K, grid):
    say(f"blk {dtype} {m}x{n} q={q} p={p} K={K} grid={grid}")
    A, _, b = _system(m, n, dtype, seed=m + n + q)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=0, q=q, alpha=1.1, max_iter=K,
                               seed=13, steps_per_exchange=p, rka_block=2, grid=grid)
    assert info.status == rka.OK and info.iterations == K
    assert st["kernel"] == 4, st
    if p:
        assert st["variant"] == p
    if grid:
        assert st["grid"] <= grid
    xo, _ = oracle.rka(A, b, q=q, alpha=1.1, max_iter=K, seed=13, dtype=_odt(dtype))
    assert_x_close(host(x), xo, what=f"blk q={q} p={st['variant']} G={st['grid']}")


def test_blk_resume_offsets_and_chunks():
    """iter_offset continues the stream; a solve split at a block boundary
    equals the whole bitwise, and any split is within 1e-12 of the oracle."""
    say("blk resume")
    A, _, b = _system(3000, 1024, seed=4)
    Ad, bd = to_dev(A), vec(b)
    kw = dict(method=0, q=16, max_iter=0, seed=21, steps_per_exchange=4, rka_block=2)

    def run(K, x0=None, off=0):
        kw.update(max_iter=K)
        return rka.solve_ex(Ad, bd, x0=x0, iter_offset=off, **kw)[0]

    full = run(40)
    assert torch.equal(full, run(40))
    half = run(12)
    assert torch.equal(full, run(28, x0=half, off=12))
    part = run(13)
    rest = run(27, x0=part, off=13)
    xo, _ = oracle.rka(A, b, q=16, max_iter=40, seed=21)
    assert_x_close(host(rest), xo, what="blk resumed off a block boundary")


@pytest.mark.parametrize("ce", [1, 5, 7, 16])
def test_blk_stops_where_the_one_iteration_kernel_stops(ce):
    """Blocks end at stopping tests: the test at iteration k sees x^(k), so the
    stopping count equals the column kernel's, and x matches the oracle's
    after that count."""
    say(f"blk stop check_every={ce}")
    A, xs, _ = _system(4000, 200, seed=5, noise=0.0)
    b = A @ xs
    Ad, bd, xd = to_dev(A), vec(b), vec(xs)
    common = dict(method=0, q=8, alpha=1.0, max_iter=200000, tol=1e-8, x_ref=xd, seed=3,
                  check_every=ce)
    x1, i1, s1 = rka.solve_ex(Ad, bd, steps_per_exchange=1, **common)
    x4, i4, s4 = rka.solve_ex(Ad, bd, steps_per_exchange=8, rka_block=2, **common)
    assert s1["kernel"] == 1 and s4["kernel"] == 4
    assert i4.status == i1.status == rka.OK and i4.iterations == i1.iterations
    assert i4.iterations % ce == 0
    xo, _ = oracle.rka(A, b, q=8, alpha=1.0, max_iter=i4.iterations, seed=3)
    assert_x_close(host(x4), xo, what="blk stopped iterate")


@pytest.mark.parametrize("variant", ["cyclic", "blocks", "worker_alpha", "row_weight"])
def test_blk_row_orders_and_weights(variant):
    say(f"blk {variant}")
    m, n, q, K = 2400, 1000, 8, 30
    A, _, b = _system(m, n, seed=31)
    Ad, bd = to_dev(A), vec(b)
    w = oracle.row_norms(A)
    kw = dict(method=0, q=q, max_iter=K, seed=17, steps_per_exchange=4, rka_block=2)
    z = np.zeros(n)
    if variant == "cyclic":
        x, info, st = rka.solve_ex(Ad, bd, sampling=2, **kw)
        xo = oracle.rka_given(A, b, z, oracle.indices_cyclic(m, 0, K, q), q=q)
    elif variant == "blocks":
        x, info, st = rka.solve_ex(Ad, bd, sampling=1, **kw)
        xo = oracle.rka_given(A, b, z, oracle.indices_blocks(w, 17, 0, K, q), q=q)
    elif variant == "worker_alpha":
        wa = np.linspace(0.6, 1.4, q)
        x, info, st = rka.solve_ex(Ad, bd, worker_alpha=vec(wa), **kw)
        xo = oracle.rka_walpha_given(A, b, z, oracle.indices(w, 17, 0, K, q), wa, q=q)
    else:
        wr = 0.5 + np.random.default_rng(3).random(m)
        x, info, st = rka.solve_ex(Ad, bd, row_weight=vec(wr), **kw)
        xo = oracle.rka_wrow_given(A, b, z, oracle.indices(w, 17, 0, K, q), wr, q=q)
    assert info.status == rka.OK and st["kernel"] == 4
    assert_x_close(host(x), xo, what=f"blk {variant}")


def test_blk_falls_back_when_blocks_do_not_fit():
    """More than 256 rows per iteration: the library runs another kernel (the
    same iteration)."""
    A, _, b = _system(3000, 1000, seed=2)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=300, max_iter=5, seed=3,
                               rka_block=2)
    assert info.status == rka.OK and st["kernel"] in (1, 2)
    xo, _ = oracle.rka(A, b, q=300, max_iter=5, seed=3)
    assert_x_close(host(x), xo, what="fallback")
    with pytest.raises(rka.RKAError):
        rka.solve_ex(to_dev(A), vec(b), method=0, q=4, max_iter=5, rka_block=3)


def test_library_chooses_blocks_with_precomputed_coefficients():
    """Left to the library (steps_per_exchange = 0, rka_block = 0), RKA on a
    shape with several workgroups runs kernel 4: several iterations per block
    up to q = 64, one iteration per block up to q = 256.  A stopping test
    every iteration, or q above 256, runs the one-iteration kernel."""
    say("blk auto selection")
    A, xs, b = _system(3000, 2000, seed=9)
    Ad, bd = to_dev(A), vec(b)
    for q, K in ((8, 24), (16, 24), (64, 24), (100, 9), (256, 5)):
        x, info, st = rka.solve_ex(Ad, bd, method=0, q=q, max_iter=K, seed=4)
        want_p = (lambda p: p >= 2) if q <= 64 else (lambda p: p == 1)
        assert info.status == rka.OK and st["kernel"] == 4 and want_p(st["variant"]), (q, st)
        xo, _ = oracle.rka(A, b, q=q, max_iter=K, seed=4)
        assert_x_close(host(x), xo, what=f"auto q={q}")
    _, _, st = rka.solve_ex(Ad, bd, method=0, q=16, max_iter=24, seed=4, tol=1e-30,
                            x_ref=vec(xs), check_every=1)
    assert st["kernel"] == 1
    _, _, st = rka.solve_ex(Ad, bd, method=0, q=300, max_iter=4, seed=4)
    assert st["kernel"] == 1


def test_blk_across_chunks():
    """45000 iterations at q = 32 (p = 4): more than one chunk's coefficients
    (the library bounds them to 512 MiB, 43676 iterations here), so the solve
    launches the coefficient pass and the iterations twice; x within 1e-12
    of the oracle."""
    say("blk two chunks")
    A, _, b = _system(3000, 1024, seed=12)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=0, q=32, alpha=1.0, max_iter=45000,
                               seed=8, rka_block=2)
    assert info.status == rka.OK and st["kernel"] == 4 and st["iterate_launches"] == 2, st
    xo, _ = oracle.rka(A, b, q=32, alpha=1.0, max_iter=45000, seed=8)
    assert_x_close(host(x), xo, what="blk two chunks")


RKAB_CASES = [
    # m, n, dtype, q, bs, K, grid
    (2000, 1000, "f64", 16, 10, 8, 0),      # 160 rows per outer iteration
    (3000, 2000, "f64", 8, 12, 6, 0),       # the longest worker block
    (1500, 777, "f64", 6, 4, 10, 0),        # scalar path, ragged slice
    (2500, 1024, "f64", 32, 2, 9, 0),
    (1500, 4096, "f32", 16, 5, 6, 0),       # narrow storage, FP64 arithmetic
    (1500, 640, "bf16", 16, 5, 6, 0),
    (700, 48, "f64", 8, 4, 12, 2),          # two workgroups
    (2000, 1000, "f64", 16, 3, 7, 100),     # more workgroups than exchange values
    # sub-blocks of c steps per worker, every worker's iterate kept per slice
    (3000, 2000, "f64", 16, 40, 3, 0),      # 4 sub-blocks of 10
    (2000, 1200, "f64", 4, 150, 2, 0),      # 13 sub-blocks, the last shorter
    (1500, 777, "f64", 8, 30, 4, 0),        # scalar path
    (1500, 640, "bf16", 8, 25, 3, 0),
    (1500, 4096, "f32", 16, 13, 3, 0),      # two sub-blocks, 7 and 6
    (700, 48, "f64", 8, 20, 5, 2),          # sub-blocks on two workgroups
    (1500, 300, "f64", 1, 40, 4, 0),        # one worker: RK over the stream, in sub-blocks
    (1500, 300, "f64", 2, 25, 4, 0),
    # slices rounded up to a whole team of lanes, the last one ragged
    (3000, 5000, "f64", 16, 10, 6, 0),      # 16-vec slices (10 rounded up), the last 4
    (2000, 7000, "f64", 8, 30, 3, 0),       # sub-blocks on 16-vec slices, the last 12
    (1500, 20000, "f32", 16, 5, 4, 0),      # narrow storage, 32-vec slices (20 rounded up)
]


@pytest.mark.parametrize("m,n,dtype,q,bs,K,grid", RKAB_CASES)
def test_blk_rkab_vs_oracle(m, n, dtype, q, bs, K, grid):
    """Column-split RKAB in kernel 4: one outer iteration's q bs rows per block
    (or sub-blocks of c steps per worker, each worker's iterate kept for the
    slice), each worker's scales from M_w = (I + N_w)^-1 of its own rows
    (streaming pass), x^(k+1) the average of the workers' iterates (Sec.
    3.4.1): within 1e-12 of the oracle on the same row stream."""
    say(f"blk rkab {dtype} {m}x{n} q={q} bs={bs} K={K} grid={grid}")
    A, _, b = _system(m, n, dtype, seed=m + n + q + bs)
    x, info, st = rka.solve_ex(to_dev(A, dtype), vec(b), method=1, q=q, block_size=bs,
                               alpha=0.9, max_iter=K, seed=11, rkab_split=2, rka_block=2,
                               grid=grid)
    assert info.status == rka.OK and info.iterations == K and info.projections == K * q * bs
    assert st["kernel"] == 4 and 2 <= st["variant"] <= min(bs, 12), st
    if q * bs <= 256 and bs <= 12:  # one block per outer iteration where it fits
        assert st["variant"] == bs, st
    if grid:
        assert st["grid"] <= grid
    odt = _odt(dtype)
    idx = oracle.indices(oracle.row_norms(A, dtype=odt), 11, 0, K, q, bs)
    xo = oracle.rkab_given(A, b, np.zeros(n), idx, q=q, block_size=bs, alpha=0.9, dtype=odt)
    assert_x_close(host(x), xo, what=f"blk rkab q={q} bs={bs}")


def test_blk_rkab_falls_back_to_the_worker_kernel():
    """Column-split RKAB asked of kernel 4 (rka_block 2) where its row groups
    cannot each serve whole workers (q = 64 on 32-lane teams at n = 10000) runs
    on the worker-split kernel, says so in the stats, and is still RKAB (Sec.
    3.4.1): within 1e-12 of the oracle on the same row stream."""
    m, n, q, bs, K = 1500, 10000, 64, 10, 3
    say(f"blk rkab fallback {m}x{n} q={q} bs={bs} K={K}")
    A, _, b = _system(m, n, "f64", seed=m + n + q + bs)
    x, info, st = rka.solve_ex(to_dev(A), vec(b), method=1, q=q, block_size=bs, alpha=0.9,
                               max_iter=K, seed=11, rkab_split=2, rka_block=2)
    assert info.status == rka.OK and info.iterations == K, info
    assert st["kernel"] == 2, st
    idx = oracle.indices(oracle.row_norms(A), 11, 0, K, q, bs)
    xo = oracle.rkab_given(A, b, np.zeros(n), idx, q=q, block_size=bs, alpha=0.9)
    assert_x_close(host(x), xo, what="blk rkab fallback")


def test_blk_rkab_stops_where_the_worker_kernel_stops():
    say("blk rkab stop")
    A, xs, _ = _system(4000, 300, seed=37, noise=0.0)
    b = A @ xs
    kw = dict(method=1, q=8, block_size=6, max_iter=20000, tol=1e-8, x_ref=vec(xs),
              check_every=5, seed=3)
    x1, i1, s1 = rka.solve_ex(to_dev(A), vec(b), rkab_split=1, **kw)
    x4, i4, s4 = rka.solve_ex(to_dev(A), vec(b), rkab_split=2, rka_block=2, **kw)
    assert s1["kernel"] == 2 and s4["kernel"] == 4
    assert i1.status == i4.status == rka.OK
    assert i4.iterations == i1.iterations and i4.iterations % 5 == 0
    xo, _ = oracle.rkab(A, b, q=8, block_size=6, max_iter=i4.iterations, seed=3)
    assert_x_close(host(x4), xo, what="blk rkab stopped iterate")
    # sub-blocks: tests fall at outer iterations only
    A, xs, _ = _system(3000, 400, seed=40, noise=0.0)
    b = A @ xs
    kw = dict(method=1, q=4, block_size=90, max_iter=5000, tol=1e-9, x_ref=vec(xs),
              check_every=2, seed=5)
    x1, i1, s1 = rka.solve_ex(to_dev(A), vec(b), rkab_split=1, **kw)
    x4, i4, s4 = rka.solve_ex(to_dev(A), vec(b), rkab_split=2, rka_block=2, **kw)
    assert s1["kernel"] == 2 and s4["kernel"] == 4
    assert i1.status == i4.status == rka.OK and i4.iterations == i1.iterations
    xo, _ = oracle.rkab(A, b, q=4, block_size=90, max_iter=i4.iterations, seed=5)
    assert_x_close(host(x4), xo, what="blk rkab sub-blocks stopped iterate")


@pytest.mark.parametrize("variant", ["cyclic", "worker_alpha", "row_weight"])
def test_blk_rkab_row_orders_and_weights(variant):
    say(f"blk rkab {variant}")
    m, n, q, bs, K = 2400, 1000, 8, 5, 9
    A, _, b = _system(m, n, seed=41)
    Ad, bd = to_dev(A), vec(b)
    w = oracle.row_norms(A)
    kw = dict(method=1, q=q, block_size=bs, max_iter=K, seed=17, rkab_split=2, rka_block=2)
    z = np.zeros(n)
    if variant == "cyclic":
        x, info, st = rka.solve_ex(Ad, bd, sampling=2, **kw)
        xo = oracle.rkab_given(A, b, z, oracle.indices_cyclic(m, 0, K, q, bs), q=q, block_size=bs)
    elif variant == "worker_alpha":
        wa = np.linspace(0.6, 1.4, q)
        x, info, st = rka.solve_ex(Ad, bd, worker_alpha=vec(wa), **kw)
        xo = oracle.rkab_walpha_given(A, b, z, oracle.indices(w, 17, 0, K, q, bs), wa, q=q,
                                      block_size=bs)
    else:
        wr = 0.5 + np.random.default_rng(5).random(m)
        x, info, st = rka.solve_ex(Ad, bd, row_weight=vec(wr), **kw)
        xo = oracle.rkab_wrow_given(A, b, z, oracle.indices(w, 17, 0, K, q, bs), wr, q=q,
                                    block_size=bs)
    assert info.status == rka.OK and st["kernel"] == 4
    assert_x_close(host(x), xo, what=f"blk rkab {variant}")


def test_library_chooses_blocks_for_column_split_rkab():
    """Left to the library, column-split RKAB runs kernel 4: one block per
    outer iteration where q bs <= 256 and bs <= 12 fit, else sub-blocks where
    q divides the row groups; otherwise kernel 3 (q = 12 here); rka_block = 1
    asks for kernel 3."""
    say("blk rkab auto selection")
    A, _, b = _system(2000, 1000, seed=43)
    Ad, bd = to_dev(A), vec(b)
    _, _, st = rka.solve_ex(Ad, bd, method=1, q=16, block_size=10, max_iter=4, seed=2)
    assert st["kernel"] == 4, st
    _, _, st = rka.solve_ex(Ad, bd, method=1, q=16, block_size=30, max_iter=2, seed=2)
    assert st["kernel"] == 4, st
    _, _, st = rka.solve_ex(Ad, bd, method=1, q=12, block_size=30, max_iter=2, seed=2)
    assert st["kernel"] == 3, st
    _, _, st = rka.solve_ex(Ad, bd, method=1, q=16, block_size=10, max_iter=4, seed=2,
                            rka_block=1)
    assert st["kernel"] == 3, st
