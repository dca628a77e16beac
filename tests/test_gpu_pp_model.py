"""Matrix-free ph-ph weights (rtbte_pp_model) against the FP64 oracle.

The library is given the problem without its |V3|^2 values (pp_v2 = None)
and the model the generator drew them from; every right-hand side
recomputes prefactor * |V3|^2 * delta of each ph-ph channel in FP64.  The
oracle sums the stored values.  The model itself is pinned against the
stored values on the CPU (tests/test_pp_model.py).

FP64: every row within 1e-12 of its magnitude sum.  Mixed precision: the
weight is formed in FP64 and rounded to FP32, so the mixed a priori bound
(with the context's weight rounding) and 1e-4 normwise hold.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_rows_close, rel_norm, say, to_dev, torch_cuda, weight_u
from tests.test_gpu_mixed import check_bounds
from tests.test_gpu_rhs import medium2d, random_state

pytestmark = pytest.mark.gpu

CASES = ["tiny2d", "tiny3d", "lattice2d", "medium2d"]


@functools.lru_cache(maxsize=None)
def wl_of(name):
    return medium2d() if name == "medium2d" else synth.build(name)


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(wl_of(name).problem_arrays())


def mf_problem(wl):
    return dict(wl.problem_arrays(), pp_v2=None)


@pytest.mark.parametrize("name", CASES)
def test_matrix_free_fp64_matches_oracle(name):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl, o = wl_of(name), orc(name)
    say(f"[pp_model] fp64 {name}")
    ctx = P.Context(mf_problem(wl), pp_model=wl.pp_model())
    assert ctx.counts() == o.counts()
    given = P.Context(wl.problem_arrays(), pp_model=wl.pp_model())   # values given, not read
    for seed, y in ((0, wl.y0), (1, random_state(wl, 1))):
        yd = to_dev(y)
        for parts in (4, 7, 6):
            out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.rhs(yd, out, parts)
            out2 = torch.full_like(out, float("nan"))
            given.rhs(yd, out2, parts)
            torch.cuda.synchronize()
            g = out.cpu().numpy()
            ref, S, A = o.rhs(y, parts=parts, scales=True)
            assert_rows_close(g, ref, A, 1e-12, f"{name} seed {seed} parts {parts}")
            assert np.array_equal(g, out2.cpu().numpy())


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "medium2d"])
def test_matrix_free_mixed_within_bound(name):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl, o = wl_of(name), orc(name)
    say(f"[pp_model] mixed {name}")
    ctx = P.Context(mf_problem(wl), precision=P.rtbte.MIXED, pp_model=wl.pp_model())
    for seed, y in ((0, wl.y0), (2, random_state(wl, 2))):
        for parts in (4, 7):
            out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.rhs(to_dev(y), out, parts)
            torch.cuda.synchronize()
            err = check_bounds(o, y, out.cpu().numpy(), parts, weight_u(ctx), f"{name} seed {seed} parts {parts}")
            if err is not None:
                assert err <= 1e-4, f"{name} seed {seed} parts {parts}: {err:.3e}"


def test_matrix_free_rates_match_oracle():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl, o = wl_of("medium2d"), orc("medium2d")
    say("[pp_model] rates medium2d")
    ctx = P.Context(mf_problem(wl), pp_model=wl.pp_model())
    y = random_state(wl, 3)
    for parts in (4, 7):
        out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.rates(to_dev(y), out, parts)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
        ref, mag = o.rates(y, parts, magnitude=True)
        assert np.all(np.isfinite(g)) and np.all(np.abs(g - ref) <= 1e-12 * mag + 1e-300)


def test_matrix_free_batch_equals_instances_alone():
    """Two instances of different grids and seeds, each with its own model,
    in one context: each computes bitwise as it does alone."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wls = [wl_of("tiny2d"), wl_of("medium2d")]
    say("[pp_model] batch of two")
    ctx = P.Context([mf_problem(w) for w in wls], pp_model=[w.pp_model() for w in wls])
    y = np.concatenate([random_state(w, 4) for w in wls])
    out = torch.empty((ctx.ny,), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, 7)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    for i, w in enumerate(wls):
        off, ne, nph = ctx.layout(i)
        one = P.Context(mf_problem(w), pp_model=w.pp_model())
        o1 = torch.empty((one.ny,), dtype=torch.float64, device="cuda")
        one.rhs(to_dev(y[off:off + ne + nph]), o1, 7)
        torch.cuda.synchronize()
        assert np.array_equal(g[off:off + ne + nph], o1.cpu().numpy())


def test_matrix_free_adaptive_step_replays_on_oracle():
    """A few adaptive ERK steps with matrix-free weights; the oracle replays
    the accepted steps over the stored values."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    from oracle import integrators as I
    wl, o = wl_of("medium2d"), orc("medium2d")
    say("[pp_model] adaptive steps")
    ctx = P.Context(mf_problem(wl), pp_model=wl.pp_model())
    y = to_dev(wl.y0)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    h = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    times = [0.0]
    for _ in range(6):
        ctx.step_adaptive(y, t, h, 1e9, one_step=True)
        torch.cuda.synchronize()
        times.append(t.item())
    yr = I.replay(o.rhs, wl.y0.copy(), np.diff(times))
    g = y.cpu().numpy()
    assert np.max(np.abs(g - yr)) <= 1e-12 * max(1.0, np.max(np.abs(yr)))


def test_matrix_free_rejected_where_unsupported():
    torch_cuda()
    import paper_2412_13402_amd as P
    wl = wl_of("tiny2d")
    m = wl.pp_model()
    with pytest.raises(P.RtbteError) as e:
        P.Context(mf_problem(wl), pp_model=m, tiled=1)
    assert e.value.code == P.rtbte.E_UNSUPPORTED
    with pytest.raises(P.RtbteError) as e:
        P.Context(mf_problem(wl), pp_model=m, fp64_layout=P.rtbte.F64_PLAIN)
    assert e.value.code == P.rtbte.E_UNSUPPORTED
    with pytest.raises(P.RtbteError) as e:
        P.Context(mf_problem(wl), pp_model=dict(m, n_modes=m["n_modes"] + 1))
    assert e.value.code == P.rtbte.E_INVAL
    with pytest.raises(P.RtbteError) as e:     # no values and no model
        P.Context(mf_problem(wl))
    assert e.value.code == P.rtbte.E_INVAL
