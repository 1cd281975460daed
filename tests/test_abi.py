"""The C ABI boundary on the CPU: librka.so loads, exports every function that
include/rka.h declares, and rejects invalid arguments before touching a
device (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rka.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rka\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    import paper_2401_17474_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return pkg.lib()


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("rka_solve", "rkab_solve", "rka_row_norms", "rka_prefix",
                     "rka_sample_indices", "rka_status_string", "rka_last_error", "rka_version"):
        assert required in names


def test_every_declared_symbol_is_exported(L):
    import paper_2401_17474_amd as pkg
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in _declared():
        assert name in exported, name
        assert getattr(L, name) is not None


def test_status_strings_and_version(L):
    import paper_2401_17474_amd as pkg
    for code in (pkg.OK, pkg.NOT_CONVERGED, pkg.EINVAL, pkg.EZERONORM, pkg.EDIVERGED,
                 pkg.ENOMEM, pkg.EDEVICE):
        assert L.rka_status_string(code).decode() == pkg.status_string(code)
    assert L.rka_version() >= 100


def _info():
    import paper_2401_17474_amd as pkg
    return pkg._Info()


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("kw,msg", [
    (dict(A=None), "non-null"),
    (dict(dtype=7), "dtype"),
    (dict(m=0), "m and n"),
    (dict(n=0), "m and n"),
    (dict(lda=3), "lda"),
    (dict(q=0), "q must"),
    (dict(alpha=0.0), "alpha"),
    (dict(alpha=float("inf")), "alpha"),
    (dict(max_iter=-1), "max_iter"),
    (dict(tol=-1.0), "tol"),
    (dict(tol=float("nan")), "tol"),
    (dict(iter_offset=-2), "iter_offset"),
])
def test_solve_rejects_invalid_arguments(L, kw, msg):
    import paper_2401_17474_amd as pkg
    a = dict(A=FAKE, dtype=0, m=10, n=4, lda=4, b=FAKE, x0=None, x=FAKE, q=2, alpha=1.0,
             max_iter=5, tol=0.0, seed=1, x_ref=None, iter_offset=0, check_every=1)
    a.update(kw)
    info = _info()
    st = L.rka_solve(a["A"], a["dtype"], a["m"], a["n"], a["lda"], a["b"], a["x0"], a["x"], a["q"],
                     a["alpha"], a["max_iter"], a["tol"], a["seed"], a["x_ref"], a["iter_offset"],
                     a["check_every"], None, ctypes.byref(info))
    assert st == pkg.EINVAL and info.status == pkg.EINVAL
    assert msg in L.rka_last_error().decode()


@pytest.mark.parametrize("bs", [0, 1 << 24])
def test_rkab_rejects_block_size(L, bs):
    import paper_2401_17474_amd as pkg
    info = _info()
    st = L.rkab_solve(FAKE, 0, 10, 4, 4, FAKE, None, FAKE, 2, bs, 1.0, 5, 0.0, 1, None, 0, 1,
                      None, ctypes.byref(info))
    assert st == pkg.EINVAL and "block_size" in L.rka_last_error().decode()


def test_hooks_reject_invalid_arguments(L):
    import paper_2401_17474_amd as pkg
    assert L.rka_row_norms(None, 0, 5, 5, 5, FAKE, None) == pkg.EINVAL
    assert L.rka_row_norms(FAKE, 0, 5, 5, 4, FAKE, None) == pkg.EINVAL
    assert L.rka_prefix(FAKE, 0, FAKE, None, None) == pkg.EINVAL
    assert L.rka_sample_indices(FAKE, FAKE, 5, 1, 0, 3, 0, 1, 0, FAKE, None) == pkg.EINVAL
    assert L.rka_sample_indices(FAKE, FAKE, 5, 1, 0, 3, 2, 1, 256, FAKE, None) == pkg.EINVAL


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    import paper_2401_17474_amd as pkg
    with pytest.raises(ValueError):
        pkg.rka_solve(torch.zeros(4, 3, dtype=torch.float64),
                      torch.zeros(4, dtype=torch.float64), q=2)


def test_alpha_star_is_the_minimizer_of_the_contraction_factor():
    """Eq. (6) against an independent numeric minimization of the worst-case
    one-step factor max(phi(s_min), phi(s_max)), where phi is the factor of
    the exact one-step error identity pinned in the oracle tests."""
    import numpy as np
    import paper_2401_17474_amd as pkg
    for q, smin, smax in [(2, 5e-4, 0.05), (4, 6.7e-4, 0.056), (16, 1e-3, 0.004),
                          (8, 0.01, 0.5), (64, 2e-4, 0.3), (1, 1e-3, 0.2)]:
        a = pkg.alpha_star(smin, smax, q)
        grid = np.linspace(1e-3, 2.5 * q, 400001)

        def phi(s):
            return 1 - 2 * grid * s + grid ** 2 * s / q + grid ** 2 * (1 - 1 / q) * s ** 2

        rho = np.maximum(phi(smin), phi(smax))
        best = grid[np.argmin(rho)]
        assert abs(a - best) <= 2 * (grid[1] - grid[0]) + 1e-9 * a, (q, a, best)


def test_plan_entry_points_reject_invalid_arguments(L):
    import paper_2401_17474_amd as pkg
    h = ctypes.c_void_p(123)
    assert L.rka_plan_create(None, 0, 5, 5, 5, None, ctypes.byref(h)) == pkg.EINVAL
    assert h.value is None  # cleared on failure
    assert L.rka_plan_create(FAKE, 9, 5, 5, 5, None, ctypes.byref(h)) == pkg.EINVAL
    assert L.rka_plan_create(FAKE, 0, 5, 5, 4, None, ctypes.byref(h)) == pkg.EINVAL
    assert L.rka_plan_create(FAKE, 0, 5, 5, 5, None, None) == pkg.EINVAL
    assert L.rka_plan_destroy(None) == pkg.OK
    info = _info()
    st = L.rka_plan_solve(None, FAKE, None, FAKE, 0, 2, 1, 1.0, 5, 0.0, 1, None, 0, None, None,
                          ctypes.byref(info), None)
    assert st == pkg.EINVAL and info.status == pkg.EINVAL
    assert "plan" in L.rka_last_error().decode()
    assert L.rka_plan_sample_indices(None, 1, 0, 3, 2, 1, 0, FAKE, None) == pkg.EINVAL
    assert L.rka_plan_row_norms(None, FAKE, None) == pkg.EINVAL
    assert L.rka_plan_query(None, None, None, None, None) == pkg.EINVAL
    o = pkg._RefineOpts(0, 2, 1, 0, 1.0, 10, 0, 1, 1, 1.0, 0.0)
    ri = pkg._RefineInfo()
    assert L.rka_plan_refine_solve(None, None, FAKE, None, FAKE, ctypes.byref(o), 1, None, None,
                                   None, ctypes.byref(ri)) == pkg.EINVAL


def test_alpha_star_entry_point_rejects_invalid_arguments(L):
    import paper_2401_17474_amd as pkg
    a = ctypes.c_double(1.0)
    for smin, smax, q in ((0.1, 0.05, 4), (-1e-3, 0.1, 4), (0.1, 1.5, 4), (0.1, 0.2, 0),
                          (float("nan"), 0.2, 4)):
        assert L.rka_alpha_star(smin, smax, q, ctypes.byref(a)) == pkg.EINVAL
    assert L.rka_alpha_star(0.1, 0.2, 4, None) == pkg.EINVAL
    # q = 1 is RK: alpha* = 1 whatever the spectrum (first case of Eq. (6))
    assert L.rka_alpha_star(0.01, 0.9, 1, ctypes.byref(a)) == pkg.OK and a.value == 1.0
