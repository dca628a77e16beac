"""Helpers shared by the GPU tests (they run through the C ABI of librtbte.so)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def say(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def rel_norm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def assert_rows_close(gpu, ref, A, tol=1e-12, what=""):
    """|gpu_i - ref_i| <= tol * A_i, with A_i = sum_channels |W| (|gain| + |loss|)
    the magnitude the row sum is formed from, and (unless the rows cancel to
    rounding level) the normwise relative error <= tol."""
    gpu = np.asarray(gpu)
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite output"
    d = np.abs(gpu - ref)
    bad = d > tol * A + 1e-300
    assert not bad.any(), (f"{what}: {bad.sum()} rows off; worst "
                           f"{np.max(d / np.maximum(A, 1e-300)):.3e} (tol {tol})")
    # Normwise relative error is only meaningful when the rows do not cancel
    # to rounding level (near equilibrium both sides compute rounding noise,
    # and the componentwise test above is the criterion).
    if np.linalg.norm(ref) > 1e-3 * np.linalg.norm(A):
        assert rel_norm(gpu, ref) <= tol, f"{what}: normwise {rel_norm(gpu, ref):.3e}"
