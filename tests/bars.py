"""Parity bars of the binary32 iterations, shared by the GPU tests and by the
CPU test that shows the bars reject planted mistakes.

A binary32 RKA / RKAB iteration on the GPU is compared with the oracle's
binary32 iteration on the same row stream.  Both carry binary32 rounding
errors of the same kind and size (the GPU's dot products, summed in FP64 per
workgroup and rounded once, are if anything more accurate than the oracle's
left-to-right binary32 sums), so their difference is bounded by a small
multiple of the rounding error one of them carries: the oracle's own distance
between its binary32 and its binary64 iteration on that stream.
"""
import numpy as np

U32 = 2.0 ** -24
FACTOR = 16.0   # allowed multiple of the oracle's binary32-vs-binary64 gap
FLOOR = 32.0    # in units of u32, for iterations whose rounding errors cancel


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def binary32_bar(x32_oracle, x64_oracle):
    """Norm-wise relative bar for a binary32 iterate against x32_oracle."""
    return max(FACTOR * rel(x32_oracle, x64_oracle), FLOOR * U32)


def oracle_pair(oracle, A, b, x0, idx, *, q, block_size=1, alpha=1.0, dtype=None, rkab=None):
    """The oracle's binary32 and binary64 iterations on one stream: RKA
    (Eq. (7)) for block_size 1 unless rkab is set, else RKAB (Sec. 3.4.1)."""
    if rkab is None:
        rkab = block_size > 1
    if not rkab:
        x32 = oracle.rka_f32_given(A, b, x0, idx, q=q, alpha=alpha, dtype=dtype)
        x64 = oracle.rka_given(A, b, x0, idx, q=q, alpha=alpha, dtype=dtype)
    else:
        x32 = oracle.rkab_f32_given(A, b, x0, idx, q=q, block_size=block_size, alpha=alpha,
                                    dtype=dtype)
        x64 = oracle.rkab_given(A, b, x0, idx, q=q, block_size=block_size, alpha=alpha,
                                dtype=dtype)
    return x32, x64
