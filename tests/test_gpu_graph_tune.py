"""HIP-graph replay of the step sequence and the launch-shape autotuner.

Graph replay runs the same kernels in the same order as eager launching, so
every result must be bitwise identical; the replays are interleaved with eager
work on the same context and checked after every call.  The autotuner may pick
any shape; the right-hand side must still match the oracle to 1e-12 (relative
to each row's magnitude sum) and the cache must reproduce the choice."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_dev, torch_cuda
from tests.test_gpu_integrators import coupled
from tests.test_gpu_rhs import medium2d

pytestmark = pytest.mark.gpu


def three_instances():
    probs, ys = [], []
    for i, (se, sp) in enumerate(((0.03, 0.003), (0.05, 0.002), (0.02, 0.004))):
        Pr, y0 = coupled(se, sp, seed=40 + i)
        probs.append(Pr)
        ys.append(y0)
    return probs, np.concatenate(ys)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replay_is_bitwise_eager(prec):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    probs, y0 = three_instances()
    n = len(probs)
    p = P.rtbte.FP64 if prec == "fp64" else P.rtbte.MIXED
    kw = dict(precision=p, rtol=1e-6, group_rows_el=4, group_rows_ph=8, item_channels=1024, steps_per_poll=4)
    ctx = {g: P.Context(probs, use_graph=g, **kw) for g in (0, 1)}
    dev = "cuda"
    y = {g: to_dev(y0) for g in (0, 1)}
    t = {g: torch.zeros(n, dtype=torch.float64, device=dev) for g in (0, 1)}
    h = {g: torch.full((n,), 0.1, dtype=torch.float64, device=dev) for g in (0, 1)}
    scratch = torch.empty_like(y[1])

    def same(label):
        torch.cuda.synchronize()
        for a in (y, t, h):
            assert torch.equal(a[0], a[1]), label

    for k, t_out in enumerate((4.0, 9.0, 15.0)):
        say(f"[graph] {prec} adaptive to {t_out} fs")
        for g in (0, 1):
            ctx[g].step_adaptive(y[g], t[g], h[g], t_out)
        same(f"adaptive to {t_out}")
        for g in (0, 1):                               # eager work between replays
            ctx[g].rhs(y[g], scratch, P.PART_ALL)
        torch.cuda.synchronize()
    for k in range(3):
        for g in (0, 1):
            ctx[g].step_adaptive(y[g], t[g], h[g], 1e9, one_step=True)
        same(f"one step {k}")
    say(f"[graph] {prec} RK4 and MIS")
    for g in (0, 1):
        ctx[g].step_rk4(y[g], t[g], 0.25, 13)
    same("rk4")
    assert ctx[1].graph_launches() > 0 and ctx[0].graph_launches() == 0
    assert ctx[0].stats(1) == ctx[1].stats(1)


@pytest.mark.parametrize("fast_mode", [0, 1])
def test_graph_replay_is_bitwise_eager_multirate(fast_mode):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    Pr, y0 = coupled()
    kw = dict(fast_mode=fast_mode, h_fast=0.7, fast_rtol=1e-7, fast_atol_el=1e-10, fast_atol_ph=1e-12,
              steps_per_poll=3)
    ctx = {g: P.Context(Pr, use_graph=g, **kw) for g in (0, 1)}
    y = {g: to_dev(y0) for g in (0, 1)}
    t = {g: torch.zeros(1, dtype=torch.float64, device="cuda") for g in (0, 1)}
    h = {g: torch.full((1,), 0.1, dtype=torch.float64, device="cuda") for g in (0, 1)}
    scratch = torch.empty_like(y[1])
    for t_out in (6.0, 18.0):
        say(f"[graph] MIS fast_mode {fast_mode} to {t_out} fs")
        for g in (0, 1):
            ctx[g].step_multirate(y[g], t[g], h[g], t_out, 6.0)
        torch.cuda.synchronize()
        for a in (y, t, h):
            assert torch.equal(a[0], a[1]), t_out
        for g in (0, 1):
            ctx[g].rhs(y[g], scratch, P.PART_PHPH)
        torch.cuda.synchronize()
    assert ctx[1].graph_launches() > 0
    assert ctx[0].stats() == ctx[1].stats()


def test_autotune_keeps_parity_and_caches(tmp_path):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = medium2d()
    o = oracle.Oracle(wl.problem_arrays())
    cache = str(tmp_path / "tune.txt")
    say("[tune] medium2d, tuned at create")
    ctx = P.Context(wl.problem_arrays(), tune=1, tune_cache=cache)
    src, ms = ctx.tuning_source()
    shape = ctx.tuning()
    say(f"    shape {shape}, {ms:.4f} ms per RHS")
    assert src == 1 and ms > 0
    assert shape[0] in (4, 8, 16) and shape[1] in (8, 16)
    y = np.random.default_rng(5).uniform(0.0, 1.0, wl.n_y)
    out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, P.PART_ALL)
    torch.cuda.synchronize()
    ref, S, A = o.rhs(y, scales=True)
    assert np.all(np.abs(out.cpu().numpy() - ref) <= 1e-12 * A + 1e-300)
    with open(cache) as f:
        lines = f.read().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    say("[tune] same problem again: from the cache")
    ctx2 = P.Context(wl.problem_arrays(), tune=1, tune_cache=cache)
    assert ctx2.tuning_source()[0] == 2 and ctx2.tuning() == shape
    ctx3 = P.Context(wl.problem_arrays(), precision=P.rtbte.MIXED, tune=1, tune_cache=cache)
    assert ctx3.tuning_source()[0] == 1          # another precision is another key
    with open(cache) as f:
        assert len([l for l in f.read().split("\n") if l.strip()]) == 2
