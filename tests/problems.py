"""Hand-built problems with closed-form behaviour (relaxation-time limits).

A "bath" state has no channels of its own as a destination row, so its
population never changes; a system state that scatters only against bath
states obeys a linear ODE y' = -(y - y_eq)/tau.
"""
import numpy as np

import synth


def _base(n_el, n_ph, eps, hw, sigma=0.002):
    return dict(n_el=n_el, n_ph=n_ph, n_k_total=64, n_q_total=64, eps=np.asarray(eps, float),
                hw=np.asarray(hw, float),
                eph_row=np.zeros(0, np.int32), eph_partner=np.zeros(0, np.int32),
                eph_phonon=np.zeros(0, np.int32), eph_g2=np.zeros(0),
                pp_row=np.zeros(0, np.int32), pp_a=np.zeros(0, np.int32), pp_b=np.zeros(0, np.int32),
                pp_v2=np.zeros(0), sigma_eph=sigma, sigma_pp=sigma, nsigma=5.0, hw_cut=0.001)


def pp_rta(n_sys=4, n_pairs=3, seed=0, scale=1.0):
    """Phonon rows 0..n_sys-1 decay only into bath pairs (a, b) with
    hw = hw_a + hw_b exactly (multiples of 5 meV); the absorption mismatch
    2*hw_b lies far outside the truncation.  One electron with no channels."""
    rng = np.random.default_rng(seed)
    hw, rows, a, b, v2 = [], [], [], [], []
    n_bath = 2 * n_sys * n_pairs
    hw_sys = [0.005 * (20 + 3 * i) for i in range(n_sys)]
    bath = []
    for i in range(n_sys):
        for j in range(n_pairs):
            wa = 0.005 * (5 + j)
            bath.append((i, wa, hw_sys[i] - wa))
    hw = list(hw_sys)
    for (i, wa, wb) in bath:
        ia = len(hw); hw.append(wa)
        ib = len(hw); hw.append(wb)
        rows.append(i); a.append(ia); b.append(ib); v2.append(scale * 1e-7 * np.exp(rng.normal()))
    P = _base(1, n_sys + n_bath, [0.0], hw)
    P.update(pp_row=np.array(rows, np.int32), pp_a=np.array(a, np.int32), pp_b=np.array(b, np.int32),
             pp_v2=np.array(v2))
    y0 = np.concatenate([[0.5], synth.bose_einstein(np.array(hw), 300.0)])
    y0[1:1 + n_sys] = synth.bose_einstein(np.array(hw_sys), 1500.0)   # hot system modes
    return P, y0, n_sys


def eph_rta(n_sys=4, n_pairs=3, seed=1, scale=1.0):
    """Electron rows 0..n_sys-1 emit only into bath electrons s with a bath
    phonon p, eps_r - hw_p - eps_s = 0 exactly; absorption mismatch 2*hw_p is
    far outside the truncation, so there are no phonon-side channels."""
    rng = np.random.default_rng(seed)
    eps = [0.1 + 0.01 * i for i in range(n_sys)]
    hw = []
    rows, partner, phonon, g2 = [], [], [], []
    for i in range(n_sys):
        for j in range(n_pairs):
            w = 0.005 * (8 + 2 * j)
            s = len(eps); eps.append(eps[i] - w)
            p = len(hw); hw.append(w)
            rows.append(i); partner.append(s); phonon.append(p); g2.append(scale * 1e-3 * np.exp(rng.normal()))
    P = _base(len(eps), len(hw), eps, hw)
    P.update(eph_row=np.array(rows, np.int32), eph_partner=np.array(partner, np.int32),
             eph_phonon=np.array(phonon, np.int32), eph_g2=np.array(g2))
    f = synth.fermi_dirac(np.array(eps), 300.0, 0.0)
    f[:n_sys] = 0.9
    y0 = np.concatenate([f, synth.bose_einstein(np.array(hw), 300.0)])
    return P, y0, n_sys


def linear_fit(rhs, y0, rows, delta=1.0):
    """Slope and root of y'_i as a function of y_i alone (rows listed), from
    two evaluations; used to read 1/tau and y_eq off the RHS."""
    ya = y0.copy()
    yb = y0.copy()
    yb[rows] += delta
    fa, fb = rhs(ya), rhs(yb)
    lam = (fb[rows] - fa[rows]) / delta
    yeq = ya[rows] - fa[rows] / lam
    return lam, yeq
