"""Pins of the oracle's random source, row weights and row sampler.

Everything here runs on the CPU and checks the oracle against facts fixed
outside it: published known-answer vectors, exact integer arithmetic, a
different search algorithm (linear scan) and the target distribution of
Eq. (4) (arXiv 2401.17474, Sec. 2.2) via a chi-square test.
"""
import os

import numpy as np
import pytest
from scipy import stats

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(orc, ctr, key, out):
    assert orc.philox(ctr, key) == out


def test_uniform_range_and_distribution(orc):
    u = np.array([orc.uniform(7, k, w, j) for k in range(200) for w in range(10)
                  for j in range(25)])
    assert u.min() >= 0.0 and u.max() < 1.0
    # 53-bit grid
    assert np.all(u * 2.0 ** 53 == np.floor(u * 2.0 ** 53))
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def test_uniform_streams_differ(orc):
    base = orc.uniform(1, 5, 3, 2, 0)
    others = {orc.uniform(2, 5, 3, 2, 0), orc.uniform(1, 6, 3, 2, 0), orc.uniform(1, 5, 4, 2, 0),
              orc.uniform(1, 5, 3, 3, 0), orc.uniform(1, 5, 3, 2, 1),
              orc.uniform(1, 5 + (1 << 32), 3, 2, 0)}
    assert base not in others and len(others) == 6


def test_row_norms_exact_on_integers(orc):
    g = np.random.default_rng(3)
    A = g.integers(-50, 51, size=(37, 129)).astype(np.float64)
    w = orc.row_norms(A)
    assert np.array_equal(w, (A.astype(np.int64) ** 2).sum(axis=1).astype(np.float64))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_row_norms_match_library(orc, dtype):
    A, _, _ = workloads.gaussian_system(50, 333, seed=11, dtype=dtype)
    w = orc.row_norms(A)
    Ad = workloads._widen_np(A, dtype)
    ref = np.einsum("ij,ij->i", Ad, Ad)
    assert np.max(np.abs(w - ref) / ref) < 1e-14


def test_row_norms_strided(orc):
    g = np.random.default_rng(4)
    big = g.standard_normal((20, 64))
    sub = big[:, :50]  # lda = 64
    assert np.array_equal(orc.row_norms(sub), orc.row_norms(np.ascontiguousarray(sub)))


def test_prefix_exact_and_zero_total(orc):
    w = np.array([3.0, 0.0, 5.0, 1.0, 0.0])
    c, st = orc.prefix(w)
    assert st == orc.OK and np.array_equal(c, np.cumsum(w))
    _, st = orc.prefix(np.zeros(4))
    assert st == orc.EZERONORM
    _, st = orc.prefix(np.array([1.0, np.inf]))
    assert st == orc.EZERONORM


def test_pick_row_hand_made(orc):
    w = np.array([0.0, 1.0, 0.0, 3.0, 0.0])
    c, _ = orc.prefix(w)
    assert orc.pick_row(c, w, 0.0) == 1                  # u = 0 -> first positive row
    assert orc.pick_row(c, w, 0.2499999) == 1            # t < 1
    assert orc.pick_row(c, w, 0.25) == 3                 # t = 1 = c_1, so c_3 > t
    assert orc.pick_row(c, w, 1.0 - 2.0 ** -53) == 3
    assert orc.pick_row(c, w, 1.0) == 3                  # t = W: clamp to last positive row


def test_pick_row_brute_force(orc):
    g = np.random.default_rng(5)
    w = g.exponential(size=41)
    w[g.integers(0, 41, size=10)] = 0.0
    c, _ = orc.prefix(w)
    us = np.concatenate([g.random(2000), [0.0, 1.0 - 2.0 ** -53]])
    for u in us:
        t = u * c[-1]
        lin = next(l for l in range(41) if c[l] > t)   # linear scan, a different search
        assert orc.pick_row(c, w, u) == lin
        assert w[lin] > 0


def test_sampler_chi_square(orc):
    g = np.random.default_rng(6)
    w = g.exponential(size=12)
    w[[2, 7]] = 0.0
    idx = orc.indices(w, seed=99, iter_offset=0, K=20000, q=5, bs=2)
    counts = np.bincount(idx, minlength=12)
    assert counts[2] == 0 and counts[7] == 0
    nz = w > 0
    expected = idx.size * w[nz] / w.sum()
    chi2 = ((counts[nz] - expected) ** 2 / expected).sum()
    assert stats.chi2.sf(chi2, nz.sum() - 1) > 1e-4


def test_indices_layout_and_offset(orc):
    g = np.random.default_rng(8)
    w = g.exponential(size=30)
    c, _ = orc.prefix(w)
    full = orc.indices(w, seed=3, iter_offset=0, K=6, q=4, bs=3)
    tail = orc.indices(w, seed=3, iter_offset=2, K=4, q=4, bs=3)
    assert np.array_equal(full[2 * 12:], tail)
    # element (k, w, j) is the pick of draw (k, w, j)
    for k, wk, j in [(0, 0, 0), (5, 3, 2), (2, 1, 1)]:
        u = orc.uniform(3, k, wk, j)
        assert full[(k * 4 + wk) * 3 + j] == orc.pick_row(c, w, u)
    dom1 = orc.indices(w, seed=3, iter_offset=0, K=6, q=4, bs=3, dom=1)
    assert not np.array_equal(full, dom1)


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_uniform_is_the_published_output_mapped(orc, ctr, key, out):
    """The uniform of draw (k, w, j, dom) under key `seed` is the published
    Philox4x32-10 output for counter (k_lo, k_hi, w, j | dom << 24) and key
    (seed_lo, seed_hi), mapped to [0, 1) from its first two words as
    ((out0 << 32 | out1) >> 11) * 2^-53.  This pins the counter layout and the
    53-bit mapping to the known-answer vectors, not to the oracle itself."""
    seed = key[0] | (key[1] << 32)
    k = ctr[0] | (ctr[1] << 32)
    w, j, dom = ctr[2], ctr[3] & 0xFFFFFF, ctr[3] >> 24
    want = (((out[0] << 32) | out[1]) >> 11) * 2.0 ** -53
    assert orc.uniform(seed, k, w, j, dom) == want


def test_uniform_of_the_zero_counter(orc):
    # the all-zero vector: out0 = 0x6627e8d5, out1 = 0xe169c58d, so
    # u = 0x6627e8d5e169c58d >> 11 over 2^53
    assert orc.uniform(0, 0, 0, 0, 0) == 0.3990464708489645
