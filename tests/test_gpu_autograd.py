"""GPU checks of the differentiable solve (paper_2401_17474_amd.autograd):
forward and backward against the FP64 QR oracle (oracle/lsq_grad.py), the
gradient of a 200 x 20 slice against central finite differences of the exact
least-squares map, and torch.autograd.gradcheck of the pair on a small FP64
system.  Every solve runs through the C ABI.

Bars: x within 1e-10 relative of x_LS; db (FP64) within 1e-9; dA (stored in
FP32 for FP32 A) within 1e-6 norm-wise, i.e. a few binary32 roundings."""
import numpy as np
import pytest

import workloads
from gpu_util import host, say, to_dev, vec
from oracle.lsq_grad import lsq, lsq_grad

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


def _opts(Aw, q, iters, sweeps=3, acc=1):
    from paper_2401_17474_amd.autograd import SolveOpts
    sv = np.linalg.svd(Aw, compute_uv=False)
    F = np.sum(sv ** 2)
    alpha = rka.alpha_star(sv[-1] ** 2 / F, sv[0] ** 2 / F, q)
    return SolveOpts(q=q, alpha=alpha, inner_iters=iters, range_iters=iters, sweeps=sweeps,
                     accumulate=acc, seed=3)


def _run(A, b, t, dtype, opts):
    from paper_2401_17474_amd.autograd import lsq_solve
    Ad = to_dev(A, dtype).requires_grad_(True)
    bd = vec(b).requires_grad_(True)
    x = lsq_solve(Ad, bd, opts)
    loss = torch.sum((x - vec(t)) ** 2)
    loss.backward()
    return host(x), host(Ad.grad.to(torch.float64)), host(bd.grad), Ad.grad.dtype


@pytest.mark.parametrize("m,n,dtype,q,iters", [(4000, 200, "f32", 32, 500),
                                               (3000, 150, "f64", 32, 500),
                                               (20000, 1000, "f32", 64, 1000)])
def test_forward_backward_vs_qr(m, n, dtype, q, iters):
    say(f"autograd {dtype} {m}x{n} q={q} iters={iters}")
    A, _, b = workloads.gaussian_system(m, n, seed=21, noise_var=1e-2, dtype=dtype)
    A = np.array(A)
    Aw = A.astype(np.float64)
    t = np.random.default_rng(22).standard_normal(n)
    x, dA, db, gdt = _run(A, b, t, dtype, _opts(Aw, q, iters, acc=1 if dtype == "f32" else 0))
    xl, r, lam, z, dAo, dbo = lsq_grad(Aw, b, 2.0 * (lsq(Aw, b) - t))
    assert np.linalg.norm(x - xl) <= 1e-10 * np.linalg.norm(xl)
    assert np.linalg.norm(db - dbo) <= 1e-9 * np.linalg.norm(dbo)
    assert gdt == (torch.float32 if dtype == "f32" else torch.float64)
    tol = 1e-6 if dtype == "f32" else 1e-9
    assert np.linalg.norm(dA - dAo) <= tol * np.linalg.norm(dAo)


def test_slice_gradient_vs_finite_differences():
    # the leading 200 x 20 block of the 20000 x 1000 FP32 system
    A, _, b = workloads.gaussian_system(20000, 1000, seed=21, noise_var=1e-2, dtype="f32")
    A = np.ascontiguousarray(np.array(A)[:200, :20])
    b = np.ascontiguousarray(b[:200])
    Aw = A.astype(np.float64)
    t = np.random.default_rng(23).standard_normal(20)
    _, dA, db, _ = _run(A, b, t, "f32", _opts(Aw, 16, 400, sweeps=4))

    def loss(Ap, bp):
        x = np.linalg.lstsq(Ap, bp, rcond=None)[0]
        return float(np.sum((x - t) ** 2))

    rng = np.random.default_rng(24)
    h = 1e-6
    for _ in range(20):
        i, j = rng.integers(0, 200), rng.integers(0, 20)
        Ap, Am = Aw.copy(), Aw.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (loss(Ap, b) - loss(Am, b)) / (2 * h)
        assert abs(fd - dA[i, j]) <= 1e-5 * max(1.0, abs(fd)), (i, j, fd, dA[i, j])
    for _ in range(10):
        i = rng.integers(0, 200)
        bp, bm = b.copy(), b.copy()
        bp[i] += h
        bm[i] -= h
        fd = (loss(Aw, bp) - loss(Aw, bm)) / (2 * h)
        assert abs(fd - db[i]) <= 1e-5 * max(1.0, abs(fd))


def test_gradcheck_fp64():
    from paper_2401_17474_amd.autograd import RKASolve
    A, _, b = workloads.gaussian_system(40, 6, seed=25, noise_var=1e-2)
    A = np.array(A)
    opts = _opts(A, 8, 300, sweeps=4, acc=0)
    Ad = to_dev(A).requires_grad_(True)
    bd = vec(b).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, bb: RKASolve.apply(a, bb, opts), (Ad, bd),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
