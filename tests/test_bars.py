"""The binary32 parity bars bite: on the CPU, every case of the binary32 GPU
parity tests is run through the oracle with a planted mistake -- one row of
the stream replaced, or the relaxation weight applied twice -- and the
planted iterate must fall outside the bar that the GPU result is held to.
(Mistakes are planted in the oracle's inputs only; nothing here runs on a
GPU.)"""
import numpy as np
import pytest

import oracle
import parity_cases as pc
import workloads
from bars import binary32_bar, oracle_pair, rel


def _odt(dtype):
    return "bf16" if dtype == "bf16" else None


def _wrong_row(idx, m):
    """The stream with its last draw replaced by the next row (mod m)."""
    bad = idx.copy()
    bad[-1] = (bad[-1] + 1) % m
    return bad


def _check(A, b, idx, *, q, bs, alpha, dtype, rkab):
    m, n = A.shape
    x0 = np.zeros(n)
    x32, x64 = oracle_pair(oracle, A, b, x0, idx, q=q, block_size=bs, alpha=alpha,
                           dtype=dtype, rkab=rkab)
    bar = binary32_bar(x32, x64)
    assert bar < 1e-4, bar  # the bar itself is near binary32 rounding

    def run(stream, a):
        if rkab:
            return oracle.rkab_f32_given(A, b, x0, stream, q=q, block_size=bs, alpha=a,
                                         dtype=dtype)
        return oracle.rka_f32_given(A, b, x0, stream, q=q, alpha=a, dtype=dtype)

    wrong = run(_wrong_row(idx, m), alpha)
    assert rel(wrong, x32) > 10 * bar, ("one wrong row passes", rel(wrong, x32), bar)
    a2 = alpha * alpha if alpha != 1.0 else 1.0
    if alpha != 1.0:
        twice = run(idx, a2)
        assert rel(twice, x32) > 10 * bar, ("alpha applied twice passes", rel(twice, x32), bar)


@pytest.mark.parametrize("m,n,q,K,dtype,grid,ar,alpha", pc.RKA32_CASES)
def test_rka32_bar_rejects_planted_mistakes(m, n, q, K, dtype, grid, ar, alpha):
    A, _, b = workloads.gaussian_system(m, n, seed=pc.RKA32_SEED_DATA, noise_var=0.01,
                                        dtype=dtype)
    A = np.array(A)
    idx = oracle.indices(oracle.row_norms(A, dtype=_odt(dtype)), pc.RKA32_SEED_SOLVE, 0, K, q)
    _check(A, b, idx, q=q, bs=1, alpha=alpha, dtype=_odt(dtype), rkab=False)


@pytest.mark.parametrize("m,n,q,bs,K,dtype,alpha", pc.RKAB32_CASES)
def test_rkab32_bar_rejects_planted_mistakes(m, n, q, bs, K, dtype, alpha):
    A, _, b = workloads.gaussian_system(m, n, seed=pc.RKAB32_SEED_DATA, noise_var=0.01,
                                        dtype=dtype)
    A = np.array(A)
    idx = oracle.indices(oracle.row_norms(A, dtype=_odt(dtype)), pc.RKAB32_SEED_SOLVE, 0, K, q,
                         bs)
    _check(A, b, idx, q=q, bs=bs, alpha=alpha, dtype=_odt(dtype), rkab=True)


@pytest.mark.parametrize("s", range(len(pc.BATCH_SHAPES)))
def test_batch_bar_rejects_planted_mistakes(s):
    (m, n), (q, bs, tpr, K), alpha = pc.BATCH_SHAPES[s], pc.BATCH_PARAMS[s], pc.BATCH_ALPHA[s]
    A, _, b = workloads.scaled_rows_system(m, n, seed=pc.BATCH_SEED0 + s, dtype="f32")
    A = np.array(A)
    idx = oracle.indices(oracle.row_norms(A), pc.BATCH_KEY + s, 0, K, q, bs)
    _check(A, b, idx, q=q, bs=bs, alpha=alpha, dtype=None, rkab=True)


def test_shared_matrix_bar_rejects_planted_mistakes():
    m, n, nrhs, q, bs, K, dseed, key = pc.MULTI_RHS
    A, _, B = workloads.multi_rhs_system(m, n, nrhs, seed=dseed)
    idx = oracle.indices(oracle.row_norms(A), key, 0, K, q, bs)
    for r in (0, nrhs - 1):
        _check(A, B[r], idx, q=q, bs=bs, alpha=1.0, dtype=None, rkab=True)
