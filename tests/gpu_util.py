"""Helpers for the GPU tests: move seeded host inputs to the device and compare
GPU results with the oracle."""
import sys

import numpy as np

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(A, dtype="f64"):
    import torch
    if dtype == "bf16":
        return torch.from_numpy(np.ascontiguousarray(A).view(np.int16)).view(torch.bfloat16).to(DEV)
    return torch.from_numpy(np.ascontiguousarray(A)).to(DEV)


def vec(v):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to(DEV)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def assert_x_close(x_gpu, x_or, tol=1e-12, what=""):
    """FP64 parity bar: norm-wise relative difference <= tol and every element
    within tol * max|x_oracle|."""
    scale = max(np.max(np.abs(x_or)), 1e-300)
    d = np.abs(x_gpu - x_or)
    rel = np.linalg.norm(x_gpu - x_or) / max(np.linalg.norm(x_or), 1e-300)
    assert rel <= tol, f"{what}: norm-wise rel diff {rel:.3e} > {tol}"
    assert d.max() <= tol * scale, f"{what}: max elementwise diff {d.max() / scale:.3e} > {tol}"
    return rel
