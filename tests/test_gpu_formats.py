"""Channel storage at the limits of the packed layouts, on hand-built problems
with many states and few channels (random channels over the whole state
range, so the largest positions occur).

* FP64: packed 12-byte channels up to 2^19 states per instance (there the
  weights keep 42 mantissa bits), the plain 16-byte layout beyond; asking
  for the packed layout beyond the limit is an error.
* Mixed: packed 8-byte channels up to 2^20 states (13 mantissa bits there,
  rounding 2^-14), the FP16-head format beyond.
Every right-hand side is checked against the oracle with the bound of the
format in use."""
import numpy as np
import pytest

import oracle
from tests.gpu_util import say, to_dev, torch_cuda, weight_u

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U_SUB = 2.0 ** -39


def many_states(n_el, n_ph, n_eph=20000, n_pp=40000, seed=0):
    """Random e-ph and ph-ph entries whose energies are chosen to conserve
    energy within the Gaussian truncation, spread over all states."""
    rng = np.random.default_rng(seed)
    eps = rng.uniform(-1.0, 1.0, n_el)
    hw = rng.uniform(0.01, 0.2, n_ph)
    r = rng.integers(0, n_el, n_eph).astype(np.int32)
    p = rng.integers(0, n_ph, n_eph).astype(np.int32)
    # partner s with eps_s close to eps_r - hw_p (emission) via sorting
    order = np.argsort(eps)
    target = eps[r] - hw[p] + rng.normal(0, 0.005, n_eph)
    s = order[np.clip(np.searchsorted(eps[order], target), 0, n_el - 1)].astype(np.int32)
    l = rng.integers(0, n_ph, n_pp).astype(np.int32)
    a = rng.integers(0, n_ph, n_pp).astype(np.int32)
    horder = np.argsort(hw)
    tb = hw[l] - hw[a] + rng.normal(0, 0.001, n_pp)
    b = horder[np.clip(np.searchsorted(hw[horder], np.abs(tb)), 0, n_ph - 1)].astype(np.int32)
    prob = dict(n_el=n_el, n_ph=n_ph, n_k_total=4096, n_q_total=4096, eps=eps, hw=hw,
                eph_row=r, eph_partner=s, eph_phonon=p, eph_g2=np.exp(rng.normal(-3, 1, n_eph)),
                pp_row=l, pp_a=a, pp_b=b, pp_v2=np.exp(rng.normal(-9, 1, n_pp)),
                sigma_eph=0.01, sigma_pp=0.002, nsigma=6.0, hw_cut=0.0)
    y = np.concatenate([rng.uniform(0, 1, n_el), rng.uniform(0, 2, n_ph)])
    return prob, y


def check(ctx, prob, y, fp64):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    o = oracle.Oracle(prob)
    assert ctx.counts() == o.counts() and sum(o.counts()) > 1000
    out = torch.full((len(y),), float("nan"), dtype=torch.float64, device="cuda")
    ctx.rhs(to_dev(y), out, P.PART_ALL)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    ref, S, A, M, Q = o.rhs(y, scales=True, unweighted=True)
    if fp64:
        assert np.all(np.abs(g - ref) <= 1e-12 * A + 1e-300)
    else:
        assert np.all(np.abs(g - ref) <= (weight_u(ctx) + 24 * U32) * A + U_SUB * o.max_weight() * M + 1e-300)


def test_fp64_packed_at_2_19_states_and_plain_beyond():
    torch_cuda()
    import paper_2412_13402_amd as P
    n = 1 << 19
    prob, y = many_states(1000, n - 1000)
    say("[formats] FP64, 2^19 states: packed")
    ctx = P.Context(prob)
    f, b, u = ctx.weight_format()
    assert (f, b) == (-2, 12) and u == 2.0 ** -43
    check(ctx, prob, y, True)
    prob2, y2 = many_states(1000, n - 999, seed=1)
    say("[formats] FP64, 2^19 + 1 states: plain")
    ctx2 = P.Context(prob2)
    assert ctx2.weight_format() == (-1, 16, 0.0)
    check(ctx2, prob2, y2, True)
    with pytest.raises(P.RtbteError):
        P.Context(prob2, fp64_layout=P.rtbte.F64_PACKED)


def test_mixed_packed_at_2_20_states_and_f16x_beyond():
    torch_cuda()
    import paper_2412_13402_amd as P
    n = 1 << 20
    prob, y = many_states(1000, n - 1000, seed=2)
    say("[formats] mixed, 2^20 states: packed, 13 mantissa bits")
    ctx = P.Context(prob, precision=P.rtbte.MIXED)
    f, b, u = ctx.weight_format()
    assert (f, b) == (P.rtbte.W_PACK8, 8) and u == 2.0 ** -14
    check(ctx, prob, y, False)
    prob2, y2 = many_states(1000, n - 999, seed=3)
    say("[formats] mixed, 2^20 + 1 states: FP16 head and tail")
    ctx2 = P.Context(prob2, precision=P.rtbte.MIXED)
    assert ctx2.weight_format()[:2] == (P.rtbte.W_F16X, 10)
    check(ctx2, prob2, y2, False)
    with pytest.raises(P.RtbteError):
        P.Context(prob2, precision=P.rtbte.MIXED, mixed_weights=P.rtbte.W_PACK8)


@pytest.mark.parametrize("n_log2", [19, 20])
def test_fp64_check_keeps_the_fp64_layout_of_the_size(n_log2):
    """A mixed context with fp64_check keeps packed FP64 lists up to 2^19
    states and plain ones beyond; its check equals the host difference of
    the mixed right-hand side and an FP64 context's."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    n = 1 << n_log2
    prob, y = many_states(1000, n - 1000, seed=4)
    say(f"[formats] FP64 check at 2^{n_log2} states")
    cm = P.Context(prob, precision=P.rtbte.MIXED, fp64_check=1)
    cd = P.Context(prob)
    assert cd.weight_format()[0] == (-2 if n_log2 <= 19 else -1)
    yd = to_dev(y)
    gm, gd = torch.empty_like(yd), torch.empty_like(yd)
    cm.rhs(yd, gm, P.PART_ALL)
    cd.rhs(yd, gd, P.PART_ALL)
    torch.cuda.synchronize()
    a, b = gm.cpu().numpy(), gd.cpu().numpy()
    e_host = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    e = cm.check_fp64(yd)[0]
    assert abs(e - e_host) <= 1e-12 * e_host and 0 < e < 1e-3   # 13-15 mantissa bits here
