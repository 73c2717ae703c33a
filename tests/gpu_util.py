"""Helpers for the GPU tests: device round trips and error metrics."""
import math
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tol_for(n, dtype):
    """Relative L2 bound per transform: 1e-6 log2 N (complex64), 1e-13 (complex128)."""
    if dtype in ("c128", np.complex128):
        return 1e-13
    return 1e-6 * max(1.0, math.log2(n))


def rel_l2(y, ref):
    """Per-transform ||y - ref||_2 / ||ref||_2 (absolute where ref is zero)."""
    y = np.atleast_2d(y).astype(np.complex128)
    ref = np.atleast_2d(ref).astype(np.complex128)
    num = np.linalg.norm(y - ref, axis=1)
    den = np.linalg.norm(ref, axis=1)
    return np.where(den > 0, num / np.where(den > 0, den, 1), num)


def np_dtype(dtype):
    return np.complex64 if dtype in ("c64", 0) else np.complex128


def run_plan(plan, x_np, inplace=False):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(x_np)).to("cuda")
    y = x if inplace else torch.empty_like(x)
    plan.execute(x, y)
    torch.cuda.synchronize()
    return y.cpu().numpy()
