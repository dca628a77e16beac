"""GPU parity of the collision integrals (HIP library vs the FP64 oracle).

Every row of f(y) from rtbte_rhs must match the oracle to 1e-12 relative to
the row's magnitude sum, and to 1e-12 normwise.  Inputs are the seeded
synthetic workloads plus random populations; cases span many tiles, ragged
row tails, every launch shape, empty lists and multi-instance contexts.
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import assert_rows_close, say, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-12


def medium2d():
    grid = dict(dim=2, L=24, lattice=1, n_bands=2, n_modes=6, t_hop=3.09, win_lo=-10.0, win_hi=10.0,
                with_eph=1, with_pp=1, shell_eph=0.13, shell_pp=0.013, keep_eph=1.0, keep_pp=0.5,
                g2_mu=-6.5, g2_sig=1.0, v2_mu=-16.0, v2_sig=1.0)
    prob = dict(sigma_eph=0.020, sigma_pp=0.002, nsigma=6.0, hw_cut=0.001)
    return synth.generate(grid, prob, dict(T_el=4000.0, T_ph=300.0), seed=synth.MASTER_SEED + 21,
                          name="medium2d")


@functools.lru_cache(maxsize=None)
def workload(name):
    if name == "medium2d":
        return medium2d()
    return synth.build(name)


@functools.lru_cache(maxsize=None)
def oracle_of(name):
    return oracle.Oracle(workload(name).problem_arrays())


def random_state(wl, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(0.0, 1.0, wl.n_el), rng.uniform(0.0, 4.0, wl.n_ph)])


CASES = ["toy2d", "tiny2d", "tiny3d", "lattice2d", "medium2d"]


@pytest.mark.parametrize("layout", ["packed", "packed-tiled", "plain"])
@pytest.mark.parametrize("name", CASES)
def test_rhs_matches_oracle(name, layout):
    """packed: the per-item launch (the default); packed-tiled: the tiled
    launch over the same channels."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload(name)
    o = oracle_of(name)
    say(f"[rhs] {name} ({layout}) n_y={wl.n_y} entries={len(wl.eph_row)}+{len(wl.pp_row)}")
    code = P.rtbte.F64_PLAIN if layout == "plain" else P.rtbte.F64_PACKED
    ctx = P.Context(wl.problem_arrays(), fp64_layout=code, tiled=1 if layout == "packed-tiled" else 0)
    assert ctx.counts() == o.counts()
    # these grids need at most 14 position bits: packed weights are exact
    assert ctx.weight_format() == ((-1, 16, 0.0) if layout == "plain" else (-2, 12, 0.0))
    for seed, y in ((0, wl.y0), (1, random_state(wl, 1)), (2, random_state(wl, 2))):
        yd = to_dev(y)
        for parts in (1, 2, 4, 3, 7):
            out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.rhs(yd, out, parts)
            torch.cuda.synchronize()
            ref, S, A = o.rhs(y, parts=parts, scales=True)
            assert_rows_close(out.cpu().numpy(), ref, A, TOL, f"{name} seed {seed} parts {parts}")


SHAPES = [(1, 1, 0), (2, 4, 0), (4, 8, 0), (8, 16, 0), (16, 12, 0), (12, 2, 0),
          (8, 16, 1000), (16, 16, 333), (1, 16, 64), (4, 4, 10 ** 7)]


@pytest.mark.parametrize("tiled", [1, 0])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("name", ["medium2d", "tiny3d"])
def test_every_launch_shape(name, shape, tiled):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    ge, gp, ic = shape
    wl = workload(name)
    o = oracle_of(name)
    say(f"[rhs] {name} group_rows_el={ge} group_rows_ph={gp} item_channels={ic} tiled={tiled}")
    ctx = P.Context(wl.problem_arrays(), group_rows_el=ge, group_rows_ph=gp, item_channels=ic, tiled=tiled)
    assert ctx.tuning()[:2] == (ge, gp) and (ic == 0 or ctx.tuning()[2] == ic)
    assert ctx.counts() == o.counts()
    y = random_state(wl, 5)
    out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, 7)
    torch.cuda.synchronize()
    ref, S, A = o.rhs(y, parts=7, scales=True)
    assert_rows_close(out.cpu().numpy(), ref, A, TOL, f"shape {shape}")


def test_empty_lists_give_zero():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload("tiny2d")
    Pr = dict(wl.problem_arrays())
    for k in ("eph_row", "eph_partner", "eph_phonon", "pp_row", "pp_a", "pp_b"):
        Pr[k] = np.zeros(0, np.int32)
    Pr["eph_g2"] = np.zeros(0)
    Pr["pp_v2"] = np.zeros(0)
    say("[rhs] empty lists")
    ctx = P.Context(Pr)
    assert ctx.counts() == (0, 0, 0)
    out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(wl.y0), out, 7)
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == 0.0)


def test_unsorted_input_order_is_handled():
    """Entries given in a scrambled order: grouping by destination row is the
    library's job; sums may differ only by rounding."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload("tiny3d")
    Pr = dict(wl.problem_arrays())
    rng = np.random.default_rng(3)
    pe = rng.permutation(len(wl.eph_row))
    pp = rng.permutation(len(wl.pp_row))
    for k in ("eph_row", "eph_partner", "eph_phonon", "eph_g2"):
        Pr[k] = np.ascontiguousarray(Pr[k][pe])
    for k in ("pp_row", "pp_a", "pp_b", "pp_v2"):
        Pr[k] = np.ascontiguousarray(Pr[k][pp])
    say("[rhs] scrambled input order")
    ctx = P.Context(Pr)
    y = random_state(wl, 4)
    out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, 7)
    torch.cuda.synchronize()
    ref, S, A = oracle_of("tiny3d").rhs(y, parts=7, scales=True)
    assert_rows_close(out.cpu().numpy(), ref, A, TOL, "scrambled")


def test_multi_instance_context_matches_single():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    names = ["toy2d", "tiny2d", "tiny3d"]
    probs = [workload(n).problem_arrays() for n in names]
    say("[rhs] three instances in one context")
    multi = P.Context(probs, group_rows_el=4, group_rows_ph=4, item_channels=512)
    ys = [random_state(workload(n), 9 + i) for i, n in enumerate(names)]
    y = np.concatenate(ys)
    assert multi.ny == len(y)
    out = torch.full((multi.ny,), float("nan"), dtype=torch.float64, device="cuda")
    multi.rhs(to_dev(y), out, 7)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, n in enumerate(names):
        off, ne, nph = multi.layout(i)
        single = P.Context(probs[i], group_rows_el=4, group_rows_ph=4, item_channels=512)
        o1 = torch.empty((ne + nph,), dtype=torch.float64, device="cuda")
        single.rhs(to_dev(ys[i]), o1, 7)
        torch.cuda.synchronize()
        assert np.array_equal(got[off:off + ne + nph], o1.cpu().numpy())
        ref, S, A = oracle_of(n).rhs(ys[i], parts=7, scales=True)
        assert_rows_close(got[off:off + ne + nph], ref, A, TOL, f"instance {i}")
        assert multi.counts(i) == oracle_of(n).counts()


def test_rhs_is_deterministic():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload("medium2d")
    ctx = P.Context(wl.problem_arrays())
    yd = to_dev(random_state(wl, 6))
    a = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    ctx.rhs(yd, a, 7)
    ctx.rhs(yd, b, 7)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("bad", ["row", "sigma", "shape", "empty"])
def test_invalid_create_is_rejected(bad):
    torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload("tiny2d")
    Pr = dict(wl.problem_arrays())
    kw = {}
    if bad == "row":
        Pr["pp_row"] = Pr["pp_row"].copy()
        Pr["pp_row"][7] = wl.n_ph
    elif bad == "sigma":
        Pr["sigma_eph"] = -1.0
    elif bad == "empty":
        Pr.update(n_el=0, n_ph=0, eps=np.zeros(0), hw=np.zeros(0))
        for k in ("eph_row", "eph_partner", "eph_phonon", "pp_row", "pp_a", "pp_b"):
            Pr[k] = np.zeros(0, np.int32)
        Pr["eph_g2"] = Pr["pp_v2"] = np.zeros(0)
    else:
        kw["group_rows_el"] = 3
    with pytest.raises(P.RtbteError) as e:
        P.Context(Pr, **kw)
    assert e.value.code == P.rtbte.E_INVAL


def test_fp64_layouts_agree_and_reject_oversize():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload("medium2d")
    say("[rhs] packed vs plain FP64 channels")
    y = random_state(wl, 9)
    outs = []
    for code in (P.rtbte.F64_PACKED, P.rtbte.F64_PLAIN):
        ctx = P.Context(wl.problem_arrays(), fp64_layout=code)
        out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
        ctx.rhs(to_dev(y), out, 7)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    o = oracle_of("medium2d")
    ref, S, A = o.rhs(y, parts=7, scales=True)
    # exact weights in both; only the order of the lane sums differs
    assert np.all(np.abs(outs[0] - outs[1]) <= 1e-14 * A + 1e-300)
    with pytest.raises(P.RtbteError):
        P.Context(wl.problem_arrays(), fp64_layout=7)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "medium2d"])
def test_pp_fold_matches_oracle_and_unfolded(name):
    """Mirror-symmetric ph-ph lists (as generated) have their emission pairs
    stored once with twice the weight: fewer stored channels, the method's
    channel count unchanged, every row still within 1e-12 A_i of the oracle
    and of the unfolded context.  A list with one mirror weight changed is
    not folded."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = workload(name)
    o = oracle.Oracle(wl.problem_arrays())
    say(f"[rhs] ph-ph fold {name}")
    y = random_state(wl, 21)
    ref, S, A = o.rhs(y, scales=True)
    outs = {}
    for fold in (1, 0):
        ctx = P.Context(wl.problem_arrays(), pp_fold=fold)
        assert ctx.counts() == o.counts()
        st = ctx.stored_counts()
        if fold:
            assert st[:2] == o.counts()[:2] and st[2] < o.counts()[2]
        else:
            assert st == o.counts()
        out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
        ctx.rhs(to_dev(y), out, P.PART_ALL)
        torch.cuda.synchronize()
        outs[fold] = out.cpu().numpy()
        assert np.all(np.abs(outs[fold] - ref) <= 1e-12 * A + 1e-300), fold
    assert np.all(np.abs(outs[1] - outs[0]) <= 1e-12 * A + 1e-300)
    # break the symmetry of one pair: no fold, still exact
    pr = dict(wl.problem_arrays())
    v2 = pr["pp_v2"].copy()
    k = int(np.flatnonzero(pr["pp_a"] != pr["pp_b"])[0])
    v2[k] *= 1.5
    pr["pp_v2"] = v2
    ob = oracle.Oracle(pr)
    ctx = P.Context(pr)
    assert ctx.stored_counts() == ctx.counts() == ob.counts()
    out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, P.PART_ALL)
    torch.cuda.synchronize()
    refb, Sb, Ab = ob.rhs(y, scales=True)
    assert np.all(np.abs(out.cpu().numpy() - refb) <= 1e-12 * Ab + 1e-300)
