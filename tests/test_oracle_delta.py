"""Pins of the shape of the broadened delta function in the oracle.

The collision integrals of Methods Eq. (e-ph) and Eq. (ph-ph) replace energy
conservation by a Gaussian of width sigma (the printed formula is garbled;
read as delta_sigma(E) = exp(-(E/sigma)^2) / (sigma sqrt(pi)), truncated at
|E| <= nsigma sigma).  The relaxation-time pins only look at delta(0), so the
width of the Gaussian is pinned here by properties that hold for that
function and for no wider or narrower one:

* swept over a fine grid of mismatches, its sum times the spacing is the
  integral over the truncation window, erf(nsigma) (a Gaussian with a wrong
  width integrates to 1/sqrt(2), sqrt(2), ...);
* delta(sigma) / delta(0) = e^-1 and delta(2 sigma) / delta(0) = e^-4;
* one channel at a mismatch x != 0 gives the row the value written out from
  the definition.

Each of the three sums (electron side, phonon side of e-ph, ph-ph) is
probed with occupations that make the factor of the probed term exactly 1
and the other term 0, so a row is minus its prefactor times the sum of its
channels' deltas.
"""
import math

import numpy as np
import pytest

import oracle
import synth

SIGMA = 0.004      # eV
NSIG = 6.0
DX = SIGMA / 8     # trapezoid spacing of the sweep; the Gaussian is negligible at +-6 sigma
N_K = N_Q = 100


def _problem(n_el, n_ph, eps, hw):
    return dict(n_el=n_el, n_ph=n_ph, n_k_total=N_K, n_q_total=N_Q,
                eps=np.asarray(eps, float), hw=np.asarray(hw, float),
                eph_row=np.zeros(0, np.int32), eph_partner=np.zeros(0, np.int32),
                eph_phonon=np.zeros(0, np.int32), eph_g2=np.zeros(0),
                pp_row=np.zeros(0, np.int32), pp_a=np.zeros(0, np.int32), pp_b=np.zeros(0, np.int32),
                pp_v2=np.zeros(0), sigma_eph=SIGMA, sigma_pp=SIGMA, nsigma=NSIG, hw_cut=0.001)


def _eph_electron_side(xs, g2=1.0):
    """Electron row 0 (eps 0, f = 1) emits a phonon (hw 0.05 eV, N = 0) into
    empty partners s_j at emission mismatch x_j.  F_em = 1, F_abs = 0, and the
    absorption mismatch x_j + 0.1 eV is outside the window."""
    hw = 0.05
    eps = [0.0] + [-hw - x for x in xs]
    P = _problem(len(eps), 1, eps, [hw])
    n = len(xs)
    P.update(eph_row=np.zeros(n, np.int32), eph_partner=np.arange(1, n + 1, dtype=np.int32),
             eph_phonon=np.zeros(n, np.int32), eph_g2=np.full(n, g2))
    y = np.concatenate([[1.0], np.zeros(n), [0.0]])
    pref = 2.0 * math.pi / synth.HBAR_EV_FS / N_Q
    return P, y, 0, pref


def _eph_phonon_side(xs, g2=1.0):
    """Phonon row (hw 0.05 eV, N = 1) absorbed by a full electron r (eps 0)
    into empty partners s_j at absorption mismatch x_j: F_abs = N_p = 1.  The
    emission mismatch x_j - 0.1 eV is outside the window."""
    hw = 0.05
    eps = [0.0] + [hw - x for x in xs]
    P = _problem(len(eps), 1, eps, [hw])
    n = len(xs)
    P.update(eph_row=np.zeros(n, np.int32), eph_partner=np.arange(1, n + 1, dtype=np.int32),
             eph_phonon=np.zeros(n, np.int32), eph_g2=np.full(n, g2))
    y = np.concatenate([[1.0], np.zeros(n), [1.0]])
    pref = 4.0 * math.pi / synth.HBAR_EV_FS / N_K
    return P, y, len(eps), pref


def _pp(xs, v2=1.0):
    """Phonon row l (hw 0.1 eV, N = 1) decays into empty partners a (0.04 eV)
    and b_j (0.06 eV + x_j): G_em = 1, G_abs = 0; the absorption mismatch
    0.12 eV + x_j is outside the window."""
    hw = [0.1, 0.04] + [0.06 + x for x in xs]
    P = _problem(1, len(hw), [0.0], hw)
    n = len(xs)
    P.update(pp_row=np.zeros(n, np.int32), pp_a=np.ones(n, np.int32),
             pp_b=np.arange(2, n + 2, dtype=np.int32), pp_v2=np.full(n, v2))
    y = np.concatenate([[0.5], [1.0, 0.0], np.zeros(n)])
    pref = 36.0 * math.pi / synth.HBAR_EV_FS / N_Q
    return P, y, 1, pref


BUILDERS = {"eph_electron_side": _eph_electron_side, "eph_phonon_side": _eph_phonon_side, "ph_ph": _pp}


def _row(builder, xs, weight=1.0):
    P, y, row, pref = builder(xs, weight)
    return -oracle.Oracle(P).rhs(y)[row] / pref


@pytest.mark.parametrize("which", sorted(BUILDERS))
def test_delta_integrates_to_the_truncated_gaussian_mass(which):
    """sum_j delta(x_j) dx over a grid that runs past the truncation equals
    erf(nsigma): the normalisation and the width together."""
    xs = DX * np.arange(-64, 65)                 # +-8 sigma; kept: |x| <= 6 sigma
    total = _row(BUILDERS[which], list(xs)) * DX
    assert total == pytest.approx(math.erf(NSIG), rel=1e-12)
    # truncation: the points beyond nsigma sigma add nothing
    inner = DX * np.arange(-48, 49)
    assert _row(BUILDERS[which], list(inner)) * DX == pytest.approx(total, rel=1e-14)


@pytest.mark.parametrize("which", sorted(BUILDERS))
def test_delta_ratios_at_one_and_two_sigma(which):
    d0 = _row(BUILDERS[which], [0.0])
    d1 = _row(BUILDERS[which], [SIGMA])
    d2 = _row(BUILDERS[which], [-2.0 * SIGMA])
    assert d1 / d0 == pytest.approx(math.exp(-1.0), rel=1e-13)
    assert d2 / d0 == pytest.approx(math.exp(-4.0), rel=1e-13)
    # the peak is 1/(sigma sqrt(pi))
    assert d0 == pytest.approx(1.0 / (SIGMA * math.sqrt(math.pi)), rel=1e-14)


@pytest.mark.parametrize("which", sorted(BUILDERS))
def test_single_channel_off_resonance(which):
    """One channel at x = 1.7 sigma with weight 0.37 eV^2: the row is
    -pref * 0.37 * exp(-(x/sigma)^2) / (sigma sqrt(pi))."""
    x, m2 = 1.7 * SIGMA, 0.37
    P, y, row, pref = BUILDERS[which]([x], m2)
    got = oracle.Oracle(P).rhs(y)[row]
    want = -pref * m2 * math.exp(-(x / SIGMA) ** 2) / (SIGMA * math.sqrt(math.pi))
    assert got == pytest.approx(want, rel=1e-13)
    # just outside the truncation the channel is dropped
    P, y, row, pref = BUILDERS[which]([NSIG * SIGMA * (1 + 1e-9)], m2)
    assert oracle.Oracle(P).rhs(y)[row] == 0.0
