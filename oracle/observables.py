"""Observables of a state, written out from their definitions (test
infrastructure: the GPU library computes them in its own kernels).

* energy_average: populations averaged over the states whose energy falls
  in each bin of [e_lo, e_hi) (the Brillouin-zone averages of the carrier
  populations and of the phonon population changes the paper plots beside
  the band structure and the dispersion, Results, Fig. 1).
* mode_temperature: the effective temperature of a phonon branch, read as
  the temperature at which Bose-Einstein occupations of the branch's states
  carry the branch's energy sum hbar omega N (the paper analyses effective
  phonon temperatures in its supplement without stating the definition in
  the text).
"""
from __future__ import annotations

import numpy as np

KB_EV_PER_K = 8.617333262e-5


def energy_average(energy, pop, e_lo, e_hi, n_bins, ref=None):
    """Per bin [e_lo + k de, e_lo + (k+1) de): (count, mean pop, mean (pop - ref))."""
    energy = np.asarray(energy, float)
    pop = np.asarray(pop, float)
    de = (e_hi - e_lo) / n_bins
    inside = (energy >= e_lo) & (energy < e_hi)
    k = np.minimum(np.floor((energy[inside] - e_lo) / de).astype(np.int64), n_bins - 1)
    count = np.bincount(k, minlength=n_bins).astype(float)
    s = np.bincount(k, weights=pop[inside], minlength=n_bins)
    d = np.bincount(k, weights=(pop - np.asarray(ref, float))[inside], minlength=n_bins) if ref is not None \
        else np.zeros(n_bins)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(count > 0, s / np.maximum(count, 1), 0.0)
        mdiff = np.where(count > 0, d / np.maximum(count, 1), 0.0)
    return count, mean, mdiff


def bose_einstein_energy(hw, T):
    hw = np.asarray(hw, float)
    with np.errstate(over="ignore"):   # exp overflow at low T: the term is 0
        return float(np.sum(hw / np.expm1(hw / (KB_EV_PER_K * T))))


def mode_temperature(hw, N, mode_of, n_modes):
    """Effective temperature of each branch (0 when its energy is not positive);
    states with hbar omega <= 0 are left out."""
    from scipy.optimize import brentq
    hw = np.asarray(hw, float)
    N = np.asarray(N, float)
    mode_of = np.asarray(mode_of)
    T = np.zeros(n_modes)
    for m in range(n_modes):
        sel = (mode_of == m) & (hw > 0)
        target = float(np.sum(hw[sel] * N[sel]))
        if not target > 0:
            continue
        f = lambda lt: bose_einstein_energy(hw[sel], np.exp(lt)) - target
        T[m] = np.exp(brentq(f, np.log(1e-2), np.log(1e7), xtol=1e-15, rtol=1e-15, maxiter=500))
    return T
