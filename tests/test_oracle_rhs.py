"""Pins of the oracle's collision integrals (Methods, Eq. (e-ph), Eq. (ph-ph)).

Each test checks the oracle against something other than itself: brute-force
grid sums in the paper's notation, exact conservation laws, the zero of the
integrals at a common-temperature equilibrium, and the linear relaxation-time
limit.  A dropped term, a wrong sign or prefactor, or a swapped index fails
at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import problems


def _rng_pop(wl, seed, even_q=True):
    """Random f in (0,1) and N > 0, with N(nu,q) = N(nu,-q) when asked."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.02, 0.98, wl.n_el)
    N = rng.uniform(0.0, 3.0, wl.n_ph)
    if even_q:
        g = wl.grid
        L, dim, nm = g["L"], g["dim"], g["n_modes"]
        for q in range(wl.n_q_total):
            mq = _neg(q, L, dim)
            if mq < q:
                N[q * nm:(q + 1) * nm] = N[mq * nm:(mq + 1) * nm]
    return np.concatenate([f, N])


def _neg(q, L, dim):
    if dim == 2:
        i, j = divmod(q, L)
        return ((L - i) % L) * L + (L - j) % L
    i, j, k = q // (L * L), (q // L) % L, q % L
    return (((L - i) % L) * L + (L - j) % L) * L + (L - k) % L


@pytest.mark.parametrize("name", ["toy2d", "tiny2d", "tiny3d", "lattice2d"])
@pytest.mark.parametrize("parts", [1, 2, 4, 7])
def test_lists_match_brute_force(name, parts):
    wl, tables = synth.build(name, dense=True)
    o = oracle.Oracle(wl.problem_arrays())
    for y in (wl.y0, _rng_pop(wl, 3, even_q=False)):
        r, S, A = o.rhs(y, parts=parts, scales=True)
        b = oracle.brute_rhs(wl, tables, y, parts=parts)
        assert np.all(np.abs(r - b) <= 1e-14 * A + 1e-300), np.max(np.abs(r - b) / (A + 1e-300))
    if parts == 7 and name != "toy2d":
        assert min(o.counts()) > 0


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "toy2d"])
def test_electron_number_conservation(name):
    """sum_nk I^{e-ph} = 0 when N is even in q (pair symmetry of |g|^2)."""
    wl = synth.build(name)
    o = oracle.Oracle(wl.problem_arrays())
    y = _rng_pop(wl, 5, even_q=True)
    r, S, A = o.rhs(y, parts=1, scales=True)
    tot = r[:wl.n_el].sum()
    assert abs(tot) <= 1e-13 * A[:wl.n_el].sum()
    assert np.abs(r[:wl.n_el]).max() > 1e-6 * A[:wl.n_el].max()   # not trivially zero


def test_energy_conservation_eph_on_integer_lattice():
    """(2/N_k) sum eps I^{e-ph} + (1/N_q) sum hw I^{ph-e} = 0 (spin 2) when every
    stored channel conserves energy exactly and N is even in q."""
    wl = synth.build("lattice2d")
    o = oracle.Oracle(wl.problem_arrays())
    assert o.counts()[0] > 0
    y = _rng_pop(wl, 7, even_q=True)
    re, _, Ae = o.rhs(y, parts=1, scales=True)
    rp, _, Ap = o.rhs(y, parts=2, scales=True)
    e_el = 2.0 / wl.n_k_total * np.dot(wl.eps, re[:wl.n_el])
    e_ph = 1.0 / wl.n_q_total * np.dot(wl.hw, rp[wl.n_el:])
    scale = (2.0 / wl.n_k_total * np.dot(np.abs(wl.eps), Ae[:wl.n_el])
             + 1.0 / wl.n_q_total * np.dot(wl.hw, Ap[wl.n_el:]))
    assert abs(e_el) > 1e-6 * scale
    assert abs(e_el + e_ph) <= 1e-13 * scale


def test_energy_conservation_pp_on_integer_lattice():
    """sum hw I^{ph-ph} = 0 for any N when energy is conserved exactly by every
    stored triplet (permutation symmetry of |V3|^2; factor 2 on absorption)."""
    wl = synth.build("lattice2d")
    o = oracle.Oracle(wl.problem_arrays())
    y = _rng_pop(wl, 9, even_q=False)
    r, _, A = o.rhs(y, parts=4, scales=True)
    e = np.dot(wl.hw, r[wl.n_el:])
    scale = np.dot(wl.hw, A[wl.n_el:])
    assert abs(e) > 0 and np.abs(r).max() > 1e-6 * A.max()
    assert abs(e) <= 1e-13 * scale


def test_phonon_number_not_conserved_by_pp():
    """Three-phonon processes change the phonon number: a sanity check that
    the energy pin above is not trivially satisfied."""
    wl = synth.build("lattice2d")
    o = oracle.Oracle(wl.problem_arrays())
    r, _, A = o.rhs(_rng_pop(wl, 9, even_q=False), parts=4, scales=True)
    assert abs(r[wl.n_el:].sum()) > 1e-6 * A.sum()


@pytest.mark.parametrize("mu", [0.0, 0.05, -0.1])
def test_equilibrium_is_a_zero_of_every_integral(mu):
    """Fermi-Dirac(T, mu) and Bose-Einstein(T) at a common T make every row of
    every integral vanish on the energy-conserving lattice."""
    wl = synth.build("lattice2d")
    o = oracle.Oracle(wl.problem_arrays())
    T = 900.0
    y = np.concatenate([synth.fermi_dirac(wl.eps, T, mu), synth.bose_einstein(wl.hw, T)])
    for parts in (1, 2, 4):
        r, _, A = o.rhs(y, parts=parts, scales=True)
        assert np.all(np.abs(r) <= 1e-14 * A + 1e-300)
        assert A.max() > 0
    # ...and a different phonon temperature does not
    y2 = np.concatenate([synth.fermi_dirac(wl.eps, T, mu), synth.bose_einstein(wl.hw, 2 * T)])
    r2, _, A2 = o.rhs(y2, parts=7, scales=True)
    assert np.abs(r2).max() > 1e-3 * A2.max()


def test_pp_relaxation_time_limit():
    """A phonon that decays only into bath pairs relaxes linearly:
    N' = -W[(Na+1)(Nb+1)N - (N+1)Na Nb] is affine in N with slope
    -W(Na+Nb+1) and root Na Nb/(Na+Nb+1)."""
    P, y0, n = problems.pp_rta()
    o = oracle.Oracle(P)
    rows = np.arange(1, 1 + n)
    lam, yeq = problems.linear_fit(o.rhs, y0, rows)
    assert np.all(lam < 0)
    # affine: a third point lies on the line
    y3 = y0.copy(); y3[rows] = 2.5
    r3 = o.rhs(y3)[rows]
    assert np.allclose(r3, lam * (2.5 - yeq), rtol=1e-12, atol=0)
    # the root matches Na Nb/(Na+Nb+1) of the bath (all pairs of one row share it
    # only if they share N; here check the weighted form row by row)
    na, nb = y0[1 + P["pp_a"]], y0[1 + P["pp_b"]]
    for i in range(n):
        sel = P["pp_row"] == i
        w = P["pp_v2"][sel]                     # weights proportional to |V3|^2
        num = np.sum(w * na[sel] * nb[sel]); den = np.sum(w * (na[sel] + nb[sel] + 1))
        assert np.isclose(yeq[i], num / den, rtol=1e-10)
    # rate ratio between rows follows |V3|^2 (prefactor common to all rows)
    w_rows = np.array([np.sum(P["pp_v2"][P["pp_row"] == i] * (na[P["pp_row"] == i] + nb[P["pp_row"] == i] + 1))
                       for i in range(n)])
    assert np.allclose(lam / lam[0], w_rows / w_rows[0], rtol=1e-10)
    # absolute rate: (36 pi/hbar)(1/N_q) |V3|^2 delta(0) (N_a + N_b + 1)
    pref = 36.0 * np.pi / synth.HBAR_EV_FS / P["n_q_total"] / (P["sigma_pp"] * np.sqrt(np.pi))
    assert np.allclose(-lam, pref * w_rows, rtol=1e-12)


def test_eph_relaxation_time_limit():
    """An electron that only emits into bath states relaxes linearly:
    f' = -W[(1 + N - f_s) f - f_s N], rate (2 pi/hbar)(1/N_q)|g|^2 delta(0)(1+N-f_s)."""
    P, y0, n = problems.eph_rta()
    o = oracle.Oracle(P)
    rows = np.arange(n)
    lam, yeq = problems.linear_fit(o.rhs, y0, rows)
    n_el = P["n_el"]
    fs = y0[P["eph_partner"]]
    Np = y0[n_el + P["eph_phonon"]]
    pref = 2.0 * np.pi / synth.HBAR_EV_FS / P["n_q_total"] / (P["sigma_eph"] * np.sqrt(np.pi))
    for i in range(n):
        sel = P["eph_row"] == i
        rate = pref * np.sum(P["eph_g2"][sel] * (1 + Np[sel] - fs[sel]))
        feq = pref * np.sum(P["eph_g2"][sel] * fs[sel] * Np[sel]) / rate
        assert np.isclose(-lam[i], rate, rtol=1e-12)
        assert np.isclose(yeq[i], feq, rtol=1e-10)
    # no phonon-side channels (absorption is far off-shell): phonons are frozen
    assert o.counts()[1] == 0
    assert np.all(o.rhs(y0)[n_el:] == 0.0)


def test_frequency_cutoff_removes_channels():
    wl = synth.build("tiny2d")
    P = wl.problem_arrays()
    o1 = oracle.Oracle(P)
    P2 = dict(P); P2["hw_cut"] = 0.1
    o2 = oracle.Oracle(P2)
    r2 = o2.rhs(wl.y0)
    soft = np.where(wl.hw < 0.1)[0]
    assert np.all(r2[wl.n_el + soft] == 0.0)
    assert all(c2 < c1 for c1, c2 in zip(o1.counts(), o2.counts()))


def test_truncation_width_controls_channel_count():
    wl = synth.build("tiny2d")
    P = wl.problem_arrays()
    counts = []
    for ns in (1.0, 2.0, 5.0):
        P2 = dict(P); P2["nsigma"] = ns
        counts.append(oracle.Oracle(P2).counts())
    assert counts[0][0] < counts[1][0] < counts[2][0]
    assert counts[0][2] < counts[1][2] < counts[2][2]


@pytest.mark.parametrize("bad", ["row", "sigma", "nsigma", "phonon"])
def test_invalid_problems_are_rejected(bad):
    wl = synth.build("tiny2d")
    P = dict(wl.problem_arrays())
    if bad == "row":
        P["eph_row"] = P["eph_row"].copy(); P["eph_row"][0] = wl.n_el
    elif bad == "sigma":
        P["sigma_pp"] = 0.0
    elif bad == "nsigma":
        P["nsigma"] = -1.0
    else:
        P["pp_b"] = P["pp_b"].copy(); P["pp_b"][3] = -1
    with pytest.raises(ValueError):
        oracle.Oracle(P)


def test_sampled_rows_equal_full_rhs():
    wl = synth.build("tiny3d")
    o = oracle.Oracle(wl.problem_arrays())
    full, S, A = o.rhs(wl.y0, scales=True)
    rows = np.array([0, 5, wl.n_el - 1, wl.n_el, wl.n_y - 1, 77])
    out, S2, A2 = o.rhs_rows(wl.y0, rows)
    assert np.array_equal(out, full[rows]) and np.array_equal(A2, A[rows])


def test_rates_closed_forms_in_relaxation_time_limits():
    """Linearized rates -d(ydot_i)/d(y_i) on the two relaxation-time problems
    equal the closed forms: (36 pi/hbar)(1/N_q) sum |V3|^2 delta(0)(N_a+N_b+1)
    for the decaying phonons, (2 pi/hbar)(1/N_q) sum |g|^2 delta(0)(1+N-f_s)
    for the emitting electrons."""
    P, y0, n = problems.pp_rta()
    o = oracle.Oracle(P)
    g = o.rates(y0, parts=4)
    na, nb = y0[1 + P["pp_a"]], y0[1 + P["pp_b"]]
    pref = 36.0 * np.pi / synth.HBAR_EV_FS / P["n_q_total"] / (P["sigma_pp"] * np.sqrt(np.pi))
    for i in range(n):
        sel = P["pp_row"] == i
        assert np.isclose(g[1 + i], pref * np.sum(P["pp_v2"][sel] * (na[sel] + nb[sel] + 1)), rtol=1e-13)
    P, y0, n = problems.eph_rta()
    o = oracle.Oracle(P)
    g = o.rates(y0, parts=1)
    n_el = P["n_el"]
    fs, Np = y0[P["eph_partner"]], y0[n_el + P["eph_phonon"]]
    pref = 2.0 * np.pi / synth.HBAR_EV_FS / P["n_q_total"] / (P["sigma_eph"] * np.sqrt(np.pi))
    for i in range(n):
        sel = P["eph_row"] == i
        assert np.isclose(g[i], pref * np.sum(P["eph_g2"][sel] * (1 + Np[sel] - fs[sel])), rtol=1e-13)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "toy2d"])
def test_rates_are_the_jacobian_diagonal(name):
    """Every occupation factor is affine in the row's own population, so once
    the entries whose partner is the row's own state are dropped (e-ph
    s = r, ph-ph a = row or b = row: there the partners-fixed rate and the
    Jacobian diagonal differ by construction), the rates are the Jacobian
    diagonal, and the central difference of row i of the right-hand side in
    y_i equals them up to rounding on every row (d = 1e-4; the difference
    rounds at ~1e-16 A_i / d)."""
    wl = synth.build(name)
    P = dict(wl.problem_arrays())
    ke = P["eph_partner"] != P["eph_row"]
    kp = (P["pp_a"] != P["pp_row"]) & (P["pp_b"] != P["pp_row"])
    for k in ("eph_row", "eph_partner", "eph_phonon", "eph_g2"):
        P[k] = P[k][ke]
    for k in ("pp_row", "pp_a", "pp_b", "pp_v2"):
        P[k] = P[k][kp]
    o = oracle.Oracle(P)
    rng = np.random.default_rng(4)
    y = np.concatenate([rng.uniform(0.05, 0.95, wl.n_el), rng.uniform(0.0, 2.0, wl.n_ph)])
    d = 1e-4
    checked = 0
    for parts in (1, 2, 4):
        g = o.rates(y, parts=parts)
        A = o.rhs(y, parts=parts, scales=True)[2]
        for i in range(wl.n_y):
            if A[i] == 0.0:
                assert g[i] == 0.0
                continue
            yp, ym = y.copy(), y.copy()
            yp[i] += d; ym[i] -= d
            fd = -(o.rhs(yp, parts=parts)[i] - o.rhs(ym, parts=parts)[i]) / (2 * d)
            assert abs(fd - g[i]) <= 1e-9 * abs(g[i]) + 1e-10 * A[i], (parts, i, fd, g[i])
            checked += 1
    assert checked > 100


def test_observables_definitions():
    """Energy averages: constant populations average to the constant in every
    occupied bin, the counts add up to the states inside the range, and the
    change against the same state is zero.  Mode temperatures: Bose-Einstein
    populations at T0 give back T0; hotter populations give a higher T."""
    from oracle import observables as obs
    wl = synth.build("tiny2d")
    c, m, d = obs.energy_average(wl.eps, np.full(wl.n_el, 0.3), -5.0, 5.0, 40, ref=np.full(wl.n_el, 0.3))
    assert c.sum() == np.sum((wl.eps >= -5.0) & (wl.eps < 5.0))
    assert np.allclose(m[c > 0], 0.3, rtol=0, atol=1e-15) and np.all(d == 0.0)
    modes = np.arange(wl.n_ph) % wl.grid["n_modes"]
    for T0 in (150.0, 300.0, 1200.0):
        N = synth.bose_einstein(wl.hw, T0)
        T = obs.mode_temperature(wl.hw, N, modes, wl.grid["n_modes"])
        assert np.allclose(T, T0, rtol=1e-10)
        T2 = obs.mode_temperature(wl.hw, N * 1.1, modes, wl.grid["n_modes"])
        assert np.all(T2 > T)


def test_carrier_number_and_inversion_kept_by_the_dynamics():
    """From the (inversion-symmetric) initial state of a thinned 3D grid,
    RK4 on the full right-hand side keeps N(q) = N(-q) and f(k) = f(-k) to
    rounding and the carrier number constant: the e-ph scattering only moves
    carriers, and the time-reversal symmetry of the inputs keeps the phonon
    populations even in q."""
    from tests.test_synth import _neg
    from oracle import integrators as I
    wl = synth.build("tiny3d", keep_eph=0.6, keep_pp=0.6, keep_pp_q=0.7)
    o = oracle.Oracle(wl.problem_arrays())
    g = wl.grid
    L, dim, nm = g["L"], g["dim"], g["n_modes"]
    pinv = np.array([_neg(l // nm, L, dim) * nm + l % nm for l in range(wl.n_ph)])
    win = {(int(k), int(b)): r for r, (k, b) in enumerate(zip(wl.el_k, wl.el_band))}
    einv = np.array([win[(_neg(int(wl.el_k[r]), L, dim), int(wl.el_band[r]))] for r in range(wl.n_el)])
    y = wl.y0.copy()
    n0 = y[:wl.n_el].sum()
    for _ in range(20):
        y = I.rk4_step(o.rhs, y, 0.05)
    f, N = y[:wl.n_el], y[wl.n_el:]
    assert np.max(np.abs(N - N[pinv])) <= 1e-14 * np.max(N)
    assert np.max(np.abs(f - f[einv])) <= 1e-14
    assert abs(f.sum() - n0) <= 1e-13 * n0
    assert np.max(np.abs(N - wl.y0[wl.n_el:])) > 1e-4 * np.max(N)   # the populations did move
