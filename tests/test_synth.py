"""Synthetic-input generator: counter-based randomness, determinism and the
symmetries the conservation pins rely on."""
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    for line in open(os.path.join(GOLD, "philox4x32_10_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat_rows())
def test_philox_known_answers(ctr, key, out):
    assert list(synth.philox4x32_10(ctr, key)) == out


def test_generation_is_deterministic_and_thread_independent():
    synth.set_threads(1)
    a = synth.build("tiny2d")
    synth.set_threads(os.cpu_count() or 4)
    b = synth.build("tiny2d")
    for name in ("eps", "hw", "eph_row", "eph_partner", "eph_phonon", "eph_g2",
                 "pp_row", "pp_a", "pp_b", "pp_v2", "y0"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    c = synth.build("tiny2d", seed=12345)
    assert not np.array_equal(a.eph_g2, c.eph_g2)


def _neg(q, L, dim):
    if dim == 2:
        i, j = divmod(q, L)
        return ((L - i) % L) * L + (L - j) % L
    i, j, k = q // (L * L), (q // L) % L, q % L
    return (((L - i) % L) * L + (L - j) % L) * L + (L - k) % L


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_inversion_symmetric_frequencies(name):
    wl = synth.build(name)
    g = wl.grid
    nm = g["n_modes"]
    for q in range(wl.n_q_total):
        mq = _neg(q, g["L"], g["dim"])
        assert np.array_equal(wl.hw[q * nm:(q + 1) * nm], wl.hw[mq * nm:(mq + 1) * nm])


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d", "toy2d"])
def test_eph_pair_symmetry(name):
    """Every stored (r -> s, nu q) has its reverse (s -> r, nu -q) with the
    same |g|^2."""
    wl = synth.build(name)
    g = wl.grid
    nm = g["n_modes"]
    key = {}
    for r, s, p, v in zip(wl.eph_row, wl.eph_partner, wl.eph_phonon, wl.eph_g2):
        key[(int(r), int(s), int(p))] = v
    assert key
    for (r, s, p), v in key.items():
        q, nu = divmod(p, nm)
        rev = (s, r, _neg(q, g["L"], g["dim"]) * nm + nu)
        assert rev in key and key[rev] == v


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_pp_permutation_symmetry(name):
    """A stored (lam; a, b) implies (lam; b, a), (a; lam, b), (b; a, lam), ...
    with the same |V3|^2 (one draw per unordered triplet)."""
    wl = synth.build(name)
    key = {}
    for l, a, b, v in zip(wl.pp_row, wl.pp_a, wl.pp_b, wl.pp_v2):
        key[(int(l), int(a), int(b))] = v
    assert key
    for (l, a, b), v in key.items():
        for perm in ((l, b, a), (a, l, b), (a, b, l), (b, l, a), (b, a, l)):
            assert perm in key and key[perm] == v


def test_momentum_conservation_of_triplets():
    wl = synth.build("tiny3d")
    g = wl.grid
    L, nm = g["L"], g["n_modes"]

    def comp(q):
        return np.array([q // (L * L), (q // L) % L, q % L])
    for l, a, b in list(zip(wl.pp_row, wl.pp_a, wl.pp_b))[:5000]:
        tot = comp(l // nm) + comp(a // nm) + comp(b // nm)
        assert np.all(tot % L == 0)


def test_window_and_initial_state():
    wl = synth.build("toy2d")
    assert np.all(np.abs(wl.eps) <= 0.5)
    f0, n0 = wl.y0[:wl.n_el], wl.y0[wl.n_el:]
    assert np.all((f0 > 0) & (f0 < 1))
    assert np.all(n0 >= 0)
    # Fermi-Dirac / Bose-Einstein closed forms at a few points
    assert synth.fermi_dirac(0.0, 300.0) == 0.5
    kT = synth.KB_EV_PER_K * 300.0
    assert np.isclose(synth.fermi_dirac(kT * np.log(3.0), 300.0), 0.25, rtol=1e-15, atol=0)
    assert np.isclose(synth.bose_einstein(kT * np.log(2.0), 300.0), 1.0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_time_reversal_symmetry(name):
    """With every kind of thinning active, the stored channels are closed
    under k -> -k with the same values: (lam; a, b) implies (-lam; -a, -b)
    with the same |V3|^2, and (r -> s, nu q) implies (-r -> -s, nu -q) with
    the same |g|^2 (real crystals have this symmetry; it keeps N even in q
    and so the carrier number conserved)."""
    wl = synth.build(name, keep_eph=0.6, keep_pp=0.6, keep_pp_q=0.7)
    g = wl.grid
    L, dim, nm = g["L"], g["dim"], g["n_modes"]

    def inv_ph(l):
        q, nu = divmod(int(l), nm)
        return _neg(q, L, dim) * nm + nu
    win = {(int(k), int(b)): r for r, (k, b) in enumerate(zip(wl.el_k, wl.el_band))}

    def inv_el(r):
        return win[(_neg(int(wl.el_k[r]), L, dim), int(wl.el_band[r]))]
    pp = {(int(l), int(a), int(b)): v for l, a, b, v in zip(wl.pp_row, wl.pp_a, wl.pp_b, wl.pp_v2)}
    assert pp
    for (l, a, b), v in pp.items():
        assert pp.get((inv_ph(l), inv_ph(a), inv_ph(b))) == v
    ep = {(int(r), int(s), int(p)): v for r, s, p, v in zip(wl.eph_row, wl.eph_partner, wl.eph_phonon, wl.eph_g2)}
    assert ep
    for (r, s, p), v in ep.items():
        assert ep.get((inv_el(r), inv_el(s), inv_ph(p))) == v
