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


def row_subset_problem(prob, rows_el, rows_ph):
    """The entries of `prob` that feed the sampled destination rows: e-ph
    entries of the sampled electron rows (electron side) or of the sampled
    phonons (their ph-e channels come from these), and ph-ph entries of the
    sampled phonon rows.  The oracle over this subset gives exactly the
    sampled rows' right-hand side (every other row is incomplete), at a
    fraction of the full lists' memory.  Indices are unchanged."""
    import numpy as np
    rows_el = np.asarray(rows_el, np.int64)
    rows_ph = np.asarray(rows_ph, np.int64)
    me = np.zeros(prob["n_el"], bool)
    me[rows_el] = True
    mp = np.zeros(prob["n_ph"], bool)
    mp[rows_ph] = True
    ke = me[prob["eph_row"]] | mp[prob["eph_phonon"]]
    kp = mp[prob["pp_row"]]
    out = dict(prob)
    for k in ("eph_row", "eph_partner", "eph_phonon", "eph_g2"):
        out[k] = np.ascontiguousarray(prob[k][ke])
    for k in ("pp_row", "pp_a", "pp_b", "pp_v2"):
        out[k] = np.ascontiguousarray(prob[k][kp])
    return out


def weight_u(ctx):
    """Relative rounding of a mixed context's weights as used in its kernel:
    the stored format's bound plus the FP32 product with the block scale."""
    return ctx.weight_format()[2] + 2.0 ** -24
