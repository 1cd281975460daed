"""GPU checks of the device alpha* ingredients (rka_gemv_t, rka_spectral_bounds)
through the C ABI: A^T t against the oracle's FP64 GEMV on the transpose, and
the Lanczos extreme Ritz values against numpy's singular values -- exact (to
rounding) when the steps reach n, inside the spectrum and close at the
extremes with fewer steps; alpha* from them against alpha* from the SVD."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import host, say, to_dev, vec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rka = pytest.importorskip("paper_2401_17474_amd")

U64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rka.lib()


def _widen(A, dtype):
    return workloads.bf16_bits_to_f64(A) if dtype == "bf16" else A.astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("m,n", [(1, 1), (513, 77), (1100, 1000), (2000, 3)])
def test_gemv_t_vs_oracle(dtype, m, n):
    say(f"gemv_t {dtype} {m}x{n}")
    A, _, _ = workloads.gaussian_system(m, n, seed=3, dtype=dtype)
    A = np.array(A)
    rng = np.random.default_rng(4)
    t, c = rng.standard_normal(m), rng.standard_normal(n)
    y = host(rka.gemv_t(to_dev(A, dtype), vec(t), c=vec(c), gamma=-0.5))
    At = np.ascontiguousarray(oracle.transpose(A, dtype="bf16" if dtype == "bf16" else None))
    yo = oracle.gemv(At, t, c=c, gamma=-0.5, dtype="bf16" if dtype == "bf16" else None)
    bound = 2 * m * U64 * (np.abs(_widen(A, dtype)).T @ np.abs(t)) * 0.5 + 4 * U64 * np.abs(c)
    assert np.all(np.abs(y - yo) <= bound)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_lanczos_exact_when_steps_reach_n(dtype):
    A, _, _ = workloads.gaussian_system(400, 40, seed=5, dtype=dtype)
    A = np.array(A)
    sv = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    lo, hi, f = rka.spectral_bounds(to_dev(A, dtype), steps=40, seed=2)
    assert abs(lo - sv[-1] ** 2) <= 1e-9 * sv[0] ** 2
    assert abs(hi - sv[0] ** 2) <= 1e-9 * sv[0] ** 2
    assert abs(f - np.sum(sv ** 2)) <= 1e-12 * f


def test_lanczos_bounds_inside_and_alpha_star():
    m, n, q = 8000, 800, 64
    A, _, _ = workloads.gaussian_system(m, n, seed=6)
    A = np.array(A)
    sv = np.linalg.svd(A, compute_uv=False)
    F = np.sum(sv ** 2)
    lo, hi, f = rka.spectral_bounds(to_dev(A), steps=150, seed=3)
    # Ritz values lie inside the spectrum and are close at both ends
    assert sv[-1] ** 2 * (1 - 1e-12) <= lo <= sv[-1] ** 2 * 1.02
    assert sv[0] ** 2 * 0.999 <= hi <= sv[0] ** 2 * (1 + 1e-12)
    a_dev = rka.alpha_star(lo / f, hi / f, q)
    a_svd = rka.alpha_star(sv[-1] ** 2 / F, sv[0] ** 2 / F, q)
    assert abs(a_dev - a_svd) <= 1e-3 * a_svd


def test_spectral_errors():
    A = torch.zeros((10, 4), dtype=torch.float64, device="cuda:0")
    with pytest.raises(rka.RKAError):
        rka.spectral_bounds(A, steps=0)
