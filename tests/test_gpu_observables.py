"""Observables on the GPU against the oracle's definitions: linearized rates
(the relaxation-time rates, partners held fixed), energy-resolved averages
of the populations and effective phonon-branch temperatures.

Rates: |rate_i - oracle_i| <= 1e-12 * sum |W| (|X| + |Y|) over row i's
channels, dF/dx = X +- Y (the FP64 bound of the right-hand side, applied to
the derivative of the occupation factor).  Energy averages: counts exact,
means within 1e-13 relative to the bin's mean absolute population (only the
summation order differs).  Temperatures: within 1e-9 relative of the
oracle's root (bisection to adjacent doubles; the sums differ in order).
"""
import functools

import numpy as np
import pytest

import oracle
import synth
from oracle import observables as obs
from tests.gpu_util import say, to_dev, torch_cuda
from tests.test_gpu_rhs import medium2d, random_state

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def wl_of(name):
    return medium2d() if name == "medium2d" else synth.build(name)


@functools.lru_cache(maxsize=None)
def orc(name):
    return oracle.Oracle(wl_of(name).problem_arrays())


@pytest.mark.parametrize("name", ["toy2d", "tiny2d", "tiny3d", "medium2d"])
def test_rates_match_oracle(name):
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl, o = wl_of(name), orc(name)
    say(f"[obs] rates {name}")
    ctx = P.Context(wl.problem_arrays())
    for seed, y in ((0, wl.y0), (1, random_state(wl, 1))):
        for parts in (7, 1, 2, 4, 3):
            out = torch.full((wl.n_y,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.rates(to_dev(y), out, parts)
            torch.cuda.synchronize()
            g = out.cpu().numpy()
            ref, mag = o.rates(y, parts, magnitude=True)
            assert np.all(np.isfinite(g))
            bad = np.abs(g - ref) > 1e-12 * mag + 1e-300
            assert not bad.any(), f"{name} seed {seed} parts {parts}: {np.flatnonzero(bad)[:5]}"


def test_rates_batched_instance_matches_alone():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wls = [synth.build("tiny2d", seed=synth.MASTER_SEED + 1 + i) for i in range(3)]
    say("[obs] rates of a batch")
    ctx = P.Context([w.problem_arrays() for w in wls])
    y = np.concatenate([w.y0 for w in wls])
    out = torch.empty((ctx.ny,), dtype=torch.float64, device="cuda")
    ctx.rates(to_dev(y), out, 7)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    for i, w in enumerate(wls):
        off, ne, nph = ctx.layout(i)
        one = P.Context(w.problem_arrays())
        o1 = torch.empty((one.ny,), dtype=torch.float64, device="cuda")
        one.rates(to_dev(w.y0), o1, 7)
        torch.cuda.synchronize()
        assert np.array_equal(g[off:off + ne + nph], o1.cpu().numpy())


def test_rates_reject_mixed_context():
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    wl = wl_of("toy2d")
    ctx = P.Context(wl.problem_arrays(), precision=P.rtbte.MIXED)
    out = torch.empty((wl.n_y,), dtype=torch.float64, device="cuda")
    with pytest.raises(P.RtbteError):
        ctx.rates(to_dev(wl.y0), out, 7)


@pytest.mark.parametrize("name", ["tiny3d", "medium2d"])
def test_energy_averages_match_definition(name):
    torch_cuda()
    import paper_2412_13402_amd as P
    wl = wl_of(name)
    say(f"[obs] energy averages {name}")
    ctx = P.Context(wl.problem_arrays())
    y, yr = random_state(wl, 4), wl.y0
    dy, dyr = to_dev(y), to_dev(yr)
    ne = wl.n_el
    for phonons, energy, lo, hi, nb in ((False, wl.eps, float(wl.eps.min()) - 0.01, float(wl.eps.max()) * 0.7, 37),
                                        (True, wl.hw, 0.0, float(wl.hw.max()) + 1e-9, 23)):
        pop, ref = (y[ne:], yr[ne:]) if phonons else (y[:ne], yr[:ne])
        c, m, d = ctx.energy_average(dy, lo, hi, nb, phonons=phonons, y_ref=dyr)
        c0, m0, d0 = obs.energy_average(energy, pop, lo, hi, nb, ref=ref)
        assert np.array_equal(c, c0)
        scale = obs.energy_average(energy, np.abs(pop) + np.abs(ref), lo, hi, nb)[1]
        assert np.all(np.abs(m - m0) <= 1e-13 * scale + 1e-300)
        assert np.all(np.abs(d - d0) <= 1e-13 * scale + 1e-300)
        c1, m1, d1 = ctx.energy_average(dy, lo, hi, nb, phonons=phonons)
        assert np.array_equal(c1, c) and np.array_equal(m1, m) and np.all(d1 == 0.0)


def test_energy_average_of_a_batch_instance_and_bad_arguments():
    torch_cuda()
    import paper_2412_13402_amd as P
    wls = [synth.build("tiny2d", seed=synth.MASTER_SEED + 5 + i) for i in range(2)]
    ctx = P.Context([w.problem_arrays() for w in wls])
    y = np.concatenate([w.y0 for w in wls])
    w = wls[1]
    c, m, _ = ctx.energy_average(to_dev(y), -3.0, 3.0, 16, inst=1)
    c0, m0, _ = obs.energy_average(w.eps, w.y0[:w.n_el], -3.0, 3.0, 16)
    assert np.array_equal(c, c0) and np.allclose(m, m0, rtol=1e-13, atol=0)
    for bad in (dict(inst=2), dict(n_bins=0)):
        args = dict(e_lo=-3.0, e_hi=3.0, n_bins=16, inst=0)
        args.update(bad)
        with pytest.raises(P.RtbteError):
            ctx.energy_average(to_dev(y), **args)
    with pytest.raises(P.RtbteError):
        ctx.energy_average(to_dev(y), 1.0, 1.0, 4)


@pytest.mark.parametrize("name", ["tiny2d", "medium2d"])
def test_mode_temperatures(name):
    torch_cuda()
    import paper_2412_13402_amd as P
    wl = wl_of(name)
    nm = wl.grid["n_modes"]
    modes = np.arange(wl.n_ph) % nm
    say(f"[obs] mode temperatures {name}")
    ctx = P.Context(wl.problem_arrays())
    ne = wl.n_el
    for T0 in (120.0, 300.0, 2500.0):
        y = wl.y0.copy()
        y[ne:] = synth.bose_einstein(wl.hw, T0)
        T = ctx.mode_temperatures(to_dev(y), modes, nm)
        assert np.allclose(T, T0, rtol=1e-9, atol=0), T
    y = random_state(wl, 6)
    T = ctx.mode_temperatures(to_dev(y), modes, nm)
    T0 = obs.mode_temperature(wl.hw, y[ne:], modes, nm)
    assert np.allclose(T, T0, rtol=1e-9, atol=0), (T, T0)
    # an empty branch and an all-zero branch give 0
    y[ne:] = 0.0
    assert np.all(ctx.mode_temperatures(to_dev(y), modes, nm + 1) == 0.0)
    with pytest.raises(P.RtbteError):
        ctx.mode_temperatures(to_dev(y), modes, nm - 1)
