"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers; it holds none of the solver's
arithmetic, and both the oracle-side tests and the GPU-side tests/bench take
their inputs from it.

Recipes (arXiv 2401.17474, Sec. 3.1 describes the paper's own sets, which are
not available; these are stand-ins of the same shapes):

* ``gaussian_system``: A with iid N(0,1) entries, planted x* ~ N(0,1),
  b = A x* + e with e ~ N(0, noise_var) (``noise_var`` is a variance).
  With ``noise_var = 0`` the system is consistent.
* ``paper_rows_system``: the consistent-set recipe of Sec. 3.1 -- every row
  draws its own mean in [-5, 5] and standard deviation in [1, 20]; the
  paper draws x* from the element law, which here is the law of one
  randomly chosen row; b = A x*.  Rows are strongly coherent (non-zero
  means), which exercises non-uniform row norms.
* ``scaled_rows_system``: iid N(0,1) entries with every row rescaled by a
  log-uniform factor in [lo, hi], so that sampling by row norm is far from
  uniform.

Each generator takes ``rng`` = "numpy" (PCG64 on the host, bit-reproducible
everywhere) or "torch" (torch's generator on ``device``; used for the
multi-GB matrices where host generation would dominate).  The returned
arrays are numpy on the host for "numpy" and torch tensors for "torch".
"""
from __future__ import annotations

import numpy as np

DATA_SEED = 240117474


def _np_rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_system(m, n, *, seed=DATA_SEED, noise_var=0.0, dtype="f64", rng="numpy",
                    device="cpu"):
    """Return (A, x_star, b).  ``dtype`` is the storage type of A: "f64",
    "f32" or "bf16" -- for narrow types the problem matrix *is* the rounded
    Gaussian, and b = A x* + e is formed from the rounded values in FP64."""
    if rng == "numpy":
        g = _np_rng(seed)
        A = g.standard_normal((m, n))
        x = g.standard_normal(n)
        e = g.standard_normal(m) * np.sqrt(noise_var) if noise_var > 0 else np.zeros(m)
        A = _round_np(A, dtype)
        Ad = _widen_np(A, dtype)
        b = Ad @ x + e
        return A, x, b
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    A = torch.randn((m, n), generator=gen, device=device, dtype=torch.float64)
    x = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    e = (torch.randn(m, generator=gen, device=device, dtype=torch.float64) * noise_var ** 0.5
         if noise_var > 0 else torch.zeros(m, device=device, dtype=torch.float64))
    A = _round_torch(A, dtype)
    b = A.to(torch.float64) @ x + e
    return A, x, b


def paper_rows_system(m, n, *, seed=DATA_SEED, dtype="f64", order="drawn", rng="numpy",
                      device="cpu"):
    """Consistent system following the recipe of Sec. 3.1.

    ``order="coherent"`` stores the same rows sorted by mu_i / sigma_i, so
    that neighbouring rows are nearly parallel (the situation in which
    Sec. 2.1 finds the cyclic order slow); the system and its solution are
    unchanged, only the row order differs.  ``rng="torch"`` draws on
    ``device`` (drawn order, FP64 only) for the multi-GB shapes."""
    if rng == "torch":
        import torch
        if order != "drawn" or dtype != "f64":
            raise ValueError("the torch generator supports the drawn order in FP64 only")
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        f64 = dict(device=device, dtype=torch.float64)
        mu = torch.rand(m, generator=gen, **f64) * 10.0 - 5.0
        sd = torch.rand(m, generator=gen, **f64) * 19.0 + 1.0
        A = torch.randn((m, n), generator=gen, **f64)
        A.mul_(sd[:, None]).add_(mu[:, None])
        r = int(torch.randint(0, m, (1,), generator=gen, device=device).item())
        x = mu[r] + sd[r] * torch.randn(n, generator=gen, **f64)
        b = A @ x
        return A, x, b
    g = _np_rng(seed)
    mu = g.uniform(-5.0, 5.0, size=m)
    sd = g.uniform(1.0, 20.0, size=m)
    A = mu[:, None] + sd[:, None] * g.standard_normal((m, n))
    r = int(g.integers(0, m))
    x = mu[r] + sd[r] * g.standard_normal(n)
    if order == "coherent":
        A = A[np.argsort(mu / sd, kind="stable")]
    elif order != "drawn":
        raise ValueError(f"unknown row order {order!r}")
    A = _round_np(A, dtype)
    b = _widen_np(A, dtype) @ x
    return A, x, b


def scaled_rows_system(m, n, *, seed=DATA_SEED, lo=0.1, hi=10.0, noise_var=0.0, dtype="f64"):
    """Gaussian system with log-uniform row scales in [lo, hi] (host only)."""
    g = _np_rng(seed)
    A = g.standard_normal((m, n))
    scale = np.exp(g.uniform(np.log(lo), np.log(hi), size=m))
    A = A * scale[:, None]
    x = g.standard_normal(n)
    e = g.standard_normal(m) * np.sqrt(noise_var) if noise_var > 0 else np.zeros(m)
    A = _round_np(A, dtype)
    b = _widen_np(A, dtype) @ x + e
    return A, x, b


def batch_shapes(count, *, seed=DATA_SEED, m_range=(1000, 50000), n_range=(50, 2000),
                 ratio=4):
    """(m, n) pairs of the batching workload: m and n log-uniform in their
    ranges, redrawn until m >= ratio * n."""
    g = _np_rng(seed)
    out = []
    while len(out) < count:
        m = int(round(np.exp(g.uniform(np.log(m_range[0]), np.log(m_range[1])))))
        n = int(round(np.exp(g.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        if m >= ratio * n:
            out.append((m, n))
    return out


def multi_rhs_system(m, n, nrhs, *, seed=DATA_SEED, dtype="f32"):
    """One Gaussian A shared by nrhs planted right-hand sides: (A, X*, B) with
    X* (nrhs x n) and B = X* A^T (nrhs x m), formed from the stored values."""
    g = _np_rng(seed)
    A = _round_np(g.standard_normal((m, n)), dtype)
    X = g.standard_normal((nrhs, n))
    B = X @ _widen_np(A, dtype).T
    return A, X, B


def seeds(k, base=1):
    """Solver seeds base, base+1, ... (the paper averages over 10 seeds)."""
    return [base + i for i in range(k)]


# -- storage rounding (round-to-nearest-even) --------------------------------

def _round_np(A, dtype):
    if dtype == "f64":
        return np.ascontiguousarray(A, dtype=np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(A, dtype=np.float32)
    if dtype == "bf16":
        f = np.ascontiguousarray(A, dtype=np.float32).view(np.uint32)
        # round to nearest even on the upper 16 bits (finite inputs only)
        lsb = (f >> 16) & 1
        return ((f + 0x7FFF + lsb) >> 16).astype(np.uint16)
    raise ValueError(dtype)


def _widen_np(A, dtype):
    if dtype == "bf16":
        return (A.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return A.astype(np.float64)


def _round_torch(A, dtype):
    import torch
    if dtype == "f64":
        return A
    if dtype == "f32":
        return A.to(torch.float32)
    if dtype == "bf16":
        return A.to(torch.bfloat16)
    raise ValueError(dtype)


def bf16_bits_to_f64(U):
    """Widen bf16 bit patterns (uint16) to float64 exactly."""
    return _widen_np(np.asarray(U, dtype=np.uint16), "bf16")
