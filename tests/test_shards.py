"""Row-sharded right-hand side, emulated on one GPU.

The multi-GPU design shards the destination rows into P contiguous blocks
balanced by channel count; each GPU holds the channels of its rows and a full
replica of y, computes its rows, and the stage vectors are all-gathered.
Here each shard is a context built from the entries that feed its rows,
evaluated on the full y.  The concatenation of the shards' rows must equal the unsharded
right-hand side to rounding and the oracle to 1e-12 of the row magnitude.
"""
import numpy as np
import pytest

import synth
from tests.gpu_util import assert_rows_close, row_subset_problem, say, to_dev, torch_cuda
from tests.test_gpu_rhs import oracle_of, random_state, workload



def shard_bounds(prob, n_shards):
    """Row blocks [b_k, b_{k+1}) of y balanced by the entries each row's
    channels come from."""
    n_el, n_ph = prob["n_el"], prob["n_ph"]
    w = np.zeros(n_el + n_ph)
    np.add.at(w, prob["eph_row"], 1.0)
    np.add.at(w, n_el + prob["eph_phonon"], 1.0)
    np.add.at(w, n_el + prob["pp_row"], 1.0)
    c = np.cumsum(w)
    cuts = [int(np.searchsorted(c, c[-1] * k / n_shards)) for k in range(1, n_shards)]
    return [0] + cuts + [n_el + n_ph]


def shard_problem(prob, lo, hi):
    """The entries that feed rows [lo, hi) of y (electron rows first, then
    phonons)."""
    n_el, n_ph = prob["n_el"], prob["n_ph"]
    el = np.arange(max(lo, 0), min(hi, n_el))
    ph = np.arange(max(lo, n_el), min(hi, n_el + n_ph)) - n_el
    return row_subset_problem(prob, el, ph)


@pytest.mark.gpu
@pytest.mark.parametrize("n_shards", [2, 4, 7])
def test_sharded_rows_equal_the_whole(n_shards):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl, o = workload("medium2d"), oracle_of("medium2d")
    prob = wl.problem_arrays()
    y = random_state(wl, 9)
    yd = to_dev(y)
    say(f"[shards] medium2d in {n_shards} row shards")
    whole = P.Context(prob)
    ref_d = torch.empty_like(yd)
    whole.rhs(yd, ref_d, P.PART_ALL)
    b = shard_bounds(prob, n_shards)
    assert b == sorted(b) and len(set(b)) == len(b)
    got = np.full(wl.n_y, np.nan)
    for k in range(n_shards):
        ctx = P.Context(shard_problem(prob, b[k], b[k + 1]))
        out = torch.empty_like(yd)
        ctx.rhs(yd, out, P.PART_ALL)     # every shard reads the full replica of y
        torch.cuda.synchronize()
        got[b[k]:b[k + 1]] = out.cpu().numpy()[b[k]:b[k + 1]]
    ref = ref_d.cpu().numpy()
    r_o, S, A = o.rhs(y, scales=True)
    assert_rows_close(got, r_o, A, 1e-12, f"{n_shards} shards vs oracle")
    assert_rows_close(got, ref, A, 1e-12, f"{n_shards} shards vs unsharded")


@pytest.mark.parametrize("n_shards", [3])
def test_oracle_shards_concatenate_to_the_whole(n_shards):
    """CPU check of the shard split itself: the oracle over each shard's
    entries gives that shard's rows of the full right-hand side exactly."""
    import oracle
    wl = synth.build("tiny2d")
    prob = wl.problem_arrays()
    y = random_state(wl, 5)
    whole = oracle.Oracle(prob).rhs(y)
    b = shard_bounds(prob, n_shards)
    got = np.concatenate([oracle.Oracle(shard_problem(prob, b[k], b[k + 1])).rhs(y)[b[k]:b[k + 1]]
                          for k in range(n_shards)])
    assert np.array_equal(got, whole)
