"""GPU parity of the batching form (rka_batch_solve) through the C ABI.

Every system of a batch is the plain RKAB iteration of Sec. 3.4.1 (block
size 1: RKA, Eq. (7)) in binary32, on its own row stream (key seed + index);
each system's x is compared with the oracle's binary32 iteration on the
oracle's own index stream, which the batch's own stream equals bit for bit.
Bar: norm-wise within the binary32 bar of tests/bars.py (16 times the
oracle's binary32-vs-binary64 gap on that stream).  Right-hand sides of a
shared matrix share one stream and are compared one by one.  The captured
graph and the plain launch sequence give bitwise-identical results."""
import numpy as np
import pytest

import oracle
import parity_cases as pc
import workloads
from bars import binary32_bar, oracle_pair, rel
from gpu_util import DEV, host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

U32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


def _odt(dtype):
    return "bf16" if dtype == "bf16" else None


def _mk(shapes, dtype, params, seed0=pc.BATCH_SEED0, alphas=None):
    host_sys, systems = [], []
    for s, ((m, n), (q, bs, tpr, K)) in enumerate(zip(shapes, params)):
        A, xs, b = workloads.scaled_rows_system(m, n, seed=seed0 + s, dtype=dtype)
        A = np.array(A)
        alpha = alphas[s] if alphas else 1.0
        host_sys.append((A, xs, b, q, bs, K, alpha))
        X = torch.zeros(n, dtype=torch.float64, device=DEV)
        systems.append(rka.BatchSystem(A=to_dev(A, dtype), B=vec(b), X=X, q=q, block_size=bs,
                                       tpr=tpr, alpha=alpha, max_iter=K))
    return host_sys, systems


SHAPES, PARAMS = pc.BATCH_SHAPES, pc.BATCH_PARAMS


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_matches_oracle_per_system(dtype):
    say(f"batch {dtype}: {len(SHAPES)} systems")
    hs, systems = _mk(SHAPES, dtype, PARAMS, alphas=pc.BATCH_ALPHA)
    res, st = rka.batch_solve(systems, seed=pc.BATCH_KEY, graph=False)
    assert st["tasks"] == len(SHAPES)
    for s, ((A, xs, b, q, bs, K, alpha), S, r) in enumerate(zip(hs, systems, res)):
        assert r["iterations"] == K and (r["q"], r["block_size"]) == (q, bs)
        w = oracle.row_norms(A, dtype=_odt(dtype))
        idx = oracle.indices(w, pc.BATCH_KEY + s, 0, K, q, bs)
        xo, x64 = oracle_pair(oracle, A, b, np.zeros(A.shape[1]), idx, q=q, block_size=bs,
                              alpha=alpha, dtype=_odt(dtype), rkab=True)
        gap, bar = rel(host(S.X), xo), binary32_bar(xo, x64)
        assert gap <= bar, (s, gap, bar)


@pytest.mark.parametrize("chunk", [0, 3])
def test_batch_row_streams_bitwise(chunk):
    """Each system's row stream (key seed + i, counters (k, w, j, 0)) equals the
    oracle's bit for bit, in one chunk or in chunks of 3 iterations; and the
    keys of refinement sweep s (seed + s * 65536 + i)."""
    say(f"batch streams chunk={chunk}")
    hs, systems = _mk(SHAPES, "f32", PARAMS)
    for key in (pc.BATCH_KEY, pc.BATCH_KEY + 2 * 65536):
        got = rka.batch_sample_indices(systems, seed=key, chunk_iters=chunk)
        for s, ((A, xs, b, q, bs, K, _), idx) in enumerate(zip(hs, got)):
            want = oracle.indices(oracle.row_norms(A), key + s, 0, K, q, bs)
            assert np.array_equal(host(idx), want), s
    for S in systems:  # the hook does not iterate
        assert not torch.any(S.X)


def test_graph_is_bitwise_the_plain_sequence():
    hs, sys_a = _mk(SHAPES[:6], "f32", PARAMS[:6])
    _, sys_b = _mk(SHAPES[:6], "f32", PARAMS[:6])
    ra, sa = rka.batch_solve(sys_a, seed=3, graph=False)
    rb, sb = rka.batch_solve(sys_b, seed=3, graph=True)
    assert sb["graph"] == 1 and sa["graph"] == 0
    for a, b in zip(sys_a, sys_b):
        assert np.array_equal(host(a.X), host(b.X))
    # a second replay of the same captured work from the same start values
    for b in sys_b:
        b.X.zero_()
    rka.batch_solve(sys_b, seed=3, graph=True)
    for a, b in zip(sys_a, sys_b):
        assert np.array_equal(host(a.X), host(b.X))


@pytest.mark.parametrize("R", [0, 1, 3])
def test_shared_matrix_many_rhs(R):
    m, n, nrhs, q, bs, K, dseed, key = pc.MULTI_RHS
    say(f"multi-rhs R={R}")
    A, Xs, B = workloads.multi_rhs_system(m, n, nrhs, seed=dseed)
    X = torch.zeros((nrhs, n), dtype=torch.float64, device=DEV)
    S = rka.BatchSystem(A=to_dev(A, "f32"), B=vec(B.ravel()).view(nrhs, m), X=X, q=q,
                        block_size=bs, tpr=64, rhs_per_task=R, max_iter=K)
    res, st = rka.batch_solve([S], seed=key, graph=False)
    Rused = res[0]["rhs_per_task"]
    assert st["tasks"] == -(-nrhs // Rused)
    w = oracle.row_norms(A)
    idx = oracle.indices(w, key, 0, K, q, bs)
    Xg = host(X)
    for r in range(nrhs):
        xo, x64 = oracle_pair(oracle, A, B[r], np.zeros(n), idx, q=q, block_size=bs, rkab=True)
        assert rel(Xg[r], xo) <= binary32_bar(xo, x64), r


def test_batch_stops_at_tolerance():
    shapes = [(2000, 50), (3000, 100), (4000, 200)]
    hs, systems = [], []
    for s, (m, n) in enumerate(shapes):
        A, xs, b = workloads.scaled_rows_system(m, n, seed=200 + s, dtype="f32")
        A = np.array(A)
        hs.append((A, xs))
        systems.append(rka.BatchSystem(A=to_dev(A, "f32"), B=vec(b),
                                       X=torch.zeros(n, dtype=torch.float64, device=DEV),
                                       X_ref=vec(xs), max_iter=20000))
    res, _ = rka.batch_solve(systems, seed=5, tol=1e-4, check_every=10)
    for (A, xs), S, r in zip(hs, systems, res):
        assert r["status"] == rka.OK and r["iterations"] < 20000 and r["iterations"] % 10 == 0
        err = np.linalg.norm(host(S.X) - xs) / np.linalg.norm(xs)
        assert err <= 1e-4 and abs(err - r["rel"]) <= 1e-3 * err


def test_batch_errors():
    A = torch.zeros((10, 4), dtype=torch.float64, device=DEV)
    S = rka.BatchSystem(A=A, B=torch.zeros(10, dtype=torch.float64, device=DEV),
                        X=torch.zeros(4, dtype=torch.float64, device=DEV))
    with pytest.raises(rka.RKAError):  # FP64 storage is not batched
        rka.batch_solve([S])
    A = torch.zeros((10, 5000), dtype=torch.float32, device=DEV)
    S = rka.BatchSystem(A=A, B=torch.zeros(10, dtype=torch.float64, device=DEV),
                        X=torch.zeros(5000, dtype=torch.float64, device=DEV))
    with pytest.raises(rka.RKAError):  # n above 16 x 256
        rka.batch_solve([S])


def test_autotuner_fills_parameters_and_tuned_batch_converges():
    shapes = [(1000, 50), (1200, 60), (3000, 300), (2500, 280), (6000, 1000)]
    hs, systems = [], []
    for s, (m, n) in enumerate(shapes):
        A, xs, b = workloads.scaled_rows_system(m, n, seed=300 + s, dtype="f32")
        A = np.array(A)
        hs.append((A, xs))
        X = torch.full((n,), 7.0, dtype=torch.float64, device=DEV)
        systems.append(rka.BatchSystem(A=to_dev(A, "f32"), B=vec(b), X=X, X_ref=vec(xs),
                                       max_iter=50000))
    systems[1].block_size = 3  # a caller's choice is kept
    for S in systems[2:]:
        S.alpha = 0.0  # chosen by the tuner
    trials = rka.batch_tune(systems, seed=2)
    assert trials > 0
    for S in systems:
        assert np.all(host(S.X) == 7.0)  # untouched
        n = S.A.shape[1]
        assert S.tpr in (16, 32, 64, 128, 256) and S.tpr * 16 >= n
        W = 256 // S.tpr
        assert S.q in (1, max(1, W // 4), W) and 1 <= S.block_size <= 256
        assert S.alpha > 0 and (S.alpha == 1.0 or (S.block_size == 1 and S.q == W))
    assert systems[1].block_size == 3 and systems[0].alpha == 1.0
    # same size class, same choice
    assert (systems[2].tpr, systems[2].q) == (systems[3].tpr, systems[3].q)
    for S in systems:
        S.X.zero_()
    res, _ = rka.batch_solve(systems, seed=5, tol=1e-5, check_every=5)
    for (A, xs), S, r in zip(hs, systems, res):
        assert r["status"] == rka.OK
        assert np.linalg.norm(host(S.X) - xs) <= 1e-5 * np.linalg.norm(xs)


@pytest.mark.parametrize("graph", [False, True])
def test_each_task_keeps_its_own_stop_flag(graph):
    # the largest task (scheduled first) converges in the first chunk; the
    # others must go on for many more chunks of 5 iterations
    easy = workloads.gaussian_system(4000, 100, seed=41, dtype="f32")
    hard = [workloads.scaled_rows_system(900, 200, seed=42 + s, dtype="f32") for s in range(3)]
    systems = []
    A, xs, b = easy
    systems.append(rka.BatchSystem(A=to_dev(np.array(A), "f32"), B=vec(b),
                                   X=torch.zeros(100, dtype=torch.float64, device=DEV),
                                   X_ref=vec(xs), q=16, block_size=100, tpr=16, max_iter=400))
    for A, xs, b in hard:
        systems.append(rka.BatchSystem(A=to_dev(np.array(A), "f32"), B=vec(b),
                                       X=torch.zeros(200, dtype=torch.float64, device=DEV),
                                       X_ref=vec(xs), q=1, block_size=4, tpr=16, max_iter=3000))
    res, st = rka.batch_solve(systems, seed=3, tol=1e-2, check_every=5, chunk_iters=5,
                              graph=graph, raise_on_error=False)
    assert st["chunks"] == 600
    assert res[0]["status"] == rka.OK and res[0]["iterations"] <= 20
    for r in res[1:]:
        assert r["iterations"] > 50  # ran far past the chunk where the first task stopped


def test_batch_refinement_goes_below_the_fp32_floor():
    # one binary32 batch solve stalls near its rounding floor; FP64 refinement
    # sweeps (batch solves for the corrections) reach 1e-10 on every system
    shapes = [(1500, 120), (2500, 300), (3000, 64)]
    hs, mk = [], []
    for s, (m, n) in enumerate(shapes):
        A, xs, b = workloads.scaled_rows_system(m, n, seed=500 + s, dtype="f32")
        hs.append((np.array(A), xs, b))

    def systems():
        return [rka.BatchSystem(A=to_dev(A, "f32"), B=vec(b),
                                X=torch.zeros(A.shape[1], dtype=torch.float64, device=DEV),
                                X_ref=vec(xs), q=8, block_size=1, tpr=32, alpha=4.0,
                                max_iter=400000) for A, xs, b in hs]
    plain = systems()
    res, _ = rka.batch_solve(plain, seed=2, tol=1e-10, check_every=50, raise_on_error=False)
    assert any(r["status"] != rka.OK for r in res)  # the binary32 floor
    ref = systems()
    res, st = rka.batch_solve(ref, seed=2, tol=1e-10, check_every=50, refine_sweeps=4)
    for (A, xs, b), S, r in zip(hs, ref, res):
        assert r["status"] == rka.OK
        assert np.linalg.norm(host(S.X) - xs) <= 1e-10 * np.linalg.norm(xs)
