"""Pins of the oracle's integrators (Methods: ERK method, MRI method).

Tableaux are pinned by their order conditions in exact rational arithmetic;
the stepping code by the exact discrete solution of linear relaxation
problems; the embedded estimate by its closed form; MIS by its two reducing
special cases and its observed order.
"""
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
import synth
from oracle import integrators as I
from tests import problems

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _paper_params():
    out = {}
    for line in open(os.path.join(GOLD, "paper_parameters.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def _full_A(tab):
    S = len(tab["b"])
    return [list(r) + [Fr(0)] * (S - len(r)) for r in tab["A"]]


def _order_conditions(b, A, c, order):
    """Butcher order conditions up to `order` (trees up to order 4)."""
    S = len(b)
    Ac = [sum(A[i][j] * c[j] for j in range(S)) for i in range(S)]
    Acc = [sum(A[i][j] * c[j] ** 2 for j in range(S)) for i in range(S)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(S)) for i in range(S)]
    conds = {
        1: [(sum(b), Fr(1))],
        2: [(sum(b[i] * c[i] for i in range(S)), Fr(1, 2))],
        3: [(sum(b[i] * c[i] ** 2 for i in range(S)), Fr(1, 3)),
            (sum(b[i] * Ac[i] for i in range(S)), Fr(1, 6))],
        4: [(sum(b[i] * c[i] ** 3 for i in range(S)), Fr(1, 4)),
            (sum(b[i] * c[i] * Ac[i] for i in range(S)), Fr(1, 8)),
            (sum(b[i] * Acc[i] for i in range(S)), Fr(1, 12)),
            (sum(b[i] * AAc[i] for i in range(S)), Fr(1, 24))],
    }
    return [lhs == rhs for p in range(1, order + 1) for lhs, rhs in conds[p]]


def test_paper_parameters_in_controller_defaults():
    pp = _paper_params()
    c = I.Controls()
    assert (c.k1, c.k2, c.k3, c.order) == (pp["pid_a1"], pp["pid_a2"], pp["pid_a3"], pp["pid_order"])
    assert len(I.ZONNEVELD["b"]) == pp["erk_stages"]


def test_zonneveld_order_conditions():
    t = I.ZONNEVELD
    A = _full_A(t)
    # row sums equal c (consistency of the abscissae)
    assert all(sum(A[i]) == t["c"][i] for i in range(5))
    assert all(_order_conditions(t["b"], A, t["c"], 4))
    assert all(_order_conditions(t["bt"], A, t["c"], 3))
    assert not all(_order_conditions(t["bt"], A, t["c"], 4))   # embedding is exactly order 3


def test_rk4_and_knoth_wolke_order_conditions():
    A = _full_A(I.RK4)
    assert all(_order_conditions(I.RK4["b"], A, I.RK4["c"], 4))
    kw = I.KNOTH_WOLKE3
    A = _full_A(kw)
    assert all(sum(A[i]) == kw["c"][i] for i in range(3))
    assert all(_order_conditions(kw["b"], A, kw["c"], 3))


def test_mis_coupling_telescopes_to_base_weights():
    chat, Om = I.mis_coupling(I.KNOTH_WOLKE3)
    assert chat == [0, Fr(1, 3), Fr(3, 4), 1]
    # the slow increments of all stages add up to b (consistency, order 1)
    tot = [sum(Om[i][j] for i in range(4)) for j in range(3)]
    assert tot == I.KNOTH_WOLKE3["b"]
    # stage i's cumulative coupling equals row i of A (reduces to the ERK)
    A = _full_A(I.KNOTH_WOLKE3)
    for i in range(1, 3):
        assert [sum(Om[m][j] for m in range(i + 1)) for j in range(3)] == A[i]
    # the printed last row (b - A_{S-1}) would break consistency
    bad = [I.KNOTH_WOLKE3["b"][j] - A[1][j] for j in range(3)]
    assert [Om[1][j] + Om[2][j] + bad[j] for j in range(3)] != I.KNOTH_WOLKE3["b"]


def _stab_poly(b, A):
    """Stability polynomial coefficients of b^T (I - zA)^{-1} 1 (exact)."""
    S = len(b)
    coeffs = [Fr(1)]
    v = [Fr(1)] * S   # A^k 1
    for _ in range(S):
        coeffs.append(sum(b[i] * v[i] for i in range(S)))
        v = [sum(A[i][j] * v[j] for j in range(S)) for i in range(S)]
    return coeffs


def test_rk4_exact_discrete_solution_on_relaxation():
    """On y' = -(y - y_eq)/tau, RK4 gives y_n - y_eq = (y_0 - y_eq) R(z)^n with
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, z = -h/tau."""
    for make in (problems.pp_rta, problems.eph_rta):
        P, y0, n = make(scale=50.0)
        o = oracle.Oracle(P)
        rows = np.arange(n) + (1 if make is problems.pp_rta else 0)
        lam, yeq = problems.linear_fit(o.rhs, y0, rows)
        h = 0.4 / np.max(-lam)
        y = y0.copy()
        for _ in range(40):
            y = I.rk4_step(o.rhs, y, h)
        z = lam * h
        R = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        expect = yeq + (y0[rows] - yeq) * R ** 40
        assert np.allclose(y[rows], expect, rtol=1e-12, atol=0)
        # bath states untouched
        mask = np.ones(len(y0), bool); mask[rows] = False
        assert np.array_equal(y[mask], y0[mask])


def test_zonneveld_solution_and_lte_closed_forms():
    """Main solution R(z) = RK4 polynomial; LTE = (R(z) - Rtilde(z)) (y - y_eq)
    with both polynomials from the tableau, and R - Rtilde = -(z^4 + z^5)/24."""
    A = _full_A(I.ZONNEVELD)
    R = _stab_poly(I.ZONNEVELD["b"], A)
    Rt = _stab_poly(I.ZONNEVELD["bt"], A)
    assert R[:5] == [1, 1, Fr(1, 2), Fr(1, 6), Fr(1, 24)] and R[5] == 0
    diff = [R[i] - Rt[i] for i in range(6)]
    assert diff == [0, 0, 0, 0, Fr(-1, 24), Fr(-1, 24)]
    P, y0, n = problems.pp_rta(scale=50.0)
    o = oracle.Oracle(P)
    rows = np.arange(1, 1 + n)
    lam, yeq = problems.linear_fit(o.rhs, y0, rows)
    h = 0.7 / np.max(-lam)
    ynew, lte = I.erk_attempt(o.rhs, y0, h)
    z = lam * h
    assert np.allclose(ynew[rows] - yeq, (y0[rows] - yeq) * sum(float(R[i]) * z ** i for i in range(6)),
                       rtol=1e-12, atol=0)
    assert np.allclose(lte[rows], -(z ** 4 + z ** 5) / 24 * (y0[rows] - yeq), rtol=1e-9, atol=0)


def test_wrms_norm_definition():
    v = np.array([3.0, -4.0])
    y = np.array([1.0, 0.0])
    # w = 1/(rtol|y| + atol): (1/(0.5+1), 1/1) -> sqrt(((3/1.5)^2 + 4^2)/2)
    assert np.isclose(I.wrms(v, y, 0.5, np.array([1.0, 1.0])), np.sqrt((4.0 + 16.0) / 2), rtol=1e-15)


def test_pid_properties():
    c = I.Controls()
    # unit error history and unit error: the ratio is the safety factor
    assert I.pid_eta(1.0, 1.0, 1.0, True, False, c) == pytest.approx(c.safety, rel=1e-15)
    # scaling law in the current error: eta ~ eps^(-k1/p)
    r = I.pid_eta(0.01, 0.3, 0.2, True, False, c) / I.pid_eta(0.02, 0.3, 0.2, True, False, c)
    assert r == pytest.approx(2.0 ** (c.k1 / c.order), rel=1e-13)
    # printed form: every exponent negative -> larger past errors shrink the step
    assert I.pid_eta(0.5, 0.9, 1.0, True, False, c) < I.pid_eta(0.5, 0.1, 1.0, True, False, c)
    assert I.pid_eta(0.5, 1.0, 0.9, True, False, c) < I.pid_eta(0.5, 1.0, 0.1, True, False, c)
    # alternate sign on eps_{k-1}
    ca = I.Controls(alt_sign=True)
    assert I.pid_eta(0.5, 0.9, 1.0, True, False, ca) > I.pid_eta(0.5, 0.1, 1.0, True, False, ca)
    # growth limits and rejection band
    assert I.pid_eta(1e-30, 1.0, 1.0, True, False, c) == c.eta_max
    # below the error floor the ratio no longer grows; on the first step it may exceed eta_max
    assert I.pid_eta(1e-30, 1.0, 1.0, True, True, c) == I.pid_eta(c.eps_floor, 1.0, 1.0, True, True, c)
    assert c.eta_max < I.pid_eta(1e-30, 1.0, 1.0, True, True, c) <= c.eta_max_first
    assert I.pid_eta(1e12, 1.0, 1.0, False, False, c) == c.eta_fail_min
    assert I.pid_eta(1.01, 1.0, 1.0, False, False, c) == c.eta_fail_max
    # repeated failures: capped at eta_fail_repeat from the small_nef-th on
    assert c.small_nef == 5 and c.eta_fail_repeat == 0.3
    assert I.pid_eta(1.01, 1.0, 1.0, False, False, c, fails=c.small_nef - 1) == c.eta_fail_max
    assert I.pid_eta(1.01, 1.0, 1.0, False, False, c, fails=c.small_nef) == c.eta_fail_repeat
    assert I.pid_eta(1e12, 1.0, 1.0, False, False, c, fails=c.small_nef + 2) == c.eta_fail_min


@pytest.mark.parametrize("accepted", [True, False])
def test_pid_history_exponents(accepted):
    """Which gain multiplies which past error (Eq. (pid_controller)): with
    everything else held, doubling eps_{k-1} scales the ratio by 2^(-k2/p)
    (printed form; 2^(+k2/p) in the alternating form) and doubling eps_{k-2}
    by 2^(-k3/p), with the gains and the order the paper states.  The points
    lie inside the growth and rejection limits."""
    pp = _paper_params()
    k1, k2, k3, p = pp["pid_a1"], pp["pid_a2"], pp["pid_a3"], pp["pid_order"]
    eps = 0.5 if accepted else 8.0
    e1, e2 = 0.3, 0.4
    for alt, s2 in ((False, -1.0), (True, 1.0)):
        c = I.Controls(alt_sign=alt)
        base = I.pid_eta(eps, e1, e2, accepted, False, c)
        assert c.eta_fail_min < base < (c.eta_max if accepted else c.eta_fail_max)
        r1 = I.pid_eta(eps, 2 * e1, e2, accepted, False, c) / base
        r2 = I.pid_eta(eps, e1, 2 * e2, accepted, False, c) / base
        r0 = I.pid_eta(2 * eps if accepted else eps / 2, e1, e2, accepted, False, c) / base
        assert r1 == pytest.approx(2.0 ** (s2 * k2 / p), rel=1e-14)
        assert r2 == pytest.approx(2.0 ** (-k3 / p), rel=1e-14)
        assert r0 == pytest.approx(2.0 ** ((-k1 if accepted else k1) / p), rel=1e-14)
        # the whole ratio at one point, from the equation with the stated gains
        want = c.safety * eps ** (-k1 / p) * e1 ** (s2 * k2 / p) * e2 ** (-k3 / p)
        assert base == pytest.approx(want, rel=1e-14)


def test_adaptive_meets_tolerance_on_relaxation():
    """Global error of the adaptive ERK on a linear relaxation problem stays
    within a small multiple of the tolerance and shrinks with it."""
    P, y0, n = problems.pp_rta(scale=50.0)
    o = oracle.Oracle(P)
    rows = np.arange(1, 1 + n)
    lam, yeq = problems.linear_fit(o.rhs, y0, rows)
    T = 3.0 / np.min(-lam)
    exact = yeq + (y0[rows] - yeq) * np.exp(lam * T)
    errs = []
    for rtol in (1e-4, 1e-6, 1e-8):
        c = I.Controls(rtol=rtol, atol_ph=1e-14, atol_el=1e-14)
        a = I.Adaptive(rhs=o.rhs, atol_vec=np.full(len(y0), 1e-14), c=c)
        y, t = a.advance(y0.copy(), 0.0, T)
        assert t == T
        errs.append(np.max(np.abs(y[rows] - exact) / np.abs(exact)))
        assert errs[-1] < 50 * rtol
        assert a.n_accept > 3
    assert errs[0] > errs[1] > errs[2]


def test_adaptive_replay_reproduces_run():
    wl = synth.build("toy2d")
    o = oracle.Oracle(wl.problem_arrays())
    atol = np.concatenate([np.full(wl.n_el, 1e-9), np.full(wl.n_ph, 1e-12)])
    a = I.Adaptive(rhs=o.rhs, atol_vec=atol, c=I.Controls(rtol=1e-5))
    y, t = a.advance(wl.y0.copy(), 0.0, 20.0)
    hs = [h for (_, h, _) in a.history]
    assert abs(sum(hs) - 20.0) < 1e-12
    y2 = I.replay(o.rhs, wl.y0.copy(), hs)
    assert np.array_equal(y, y2)


def _coupled_problem(scale_eph=0.03, scale_pp=0.003):
    """tiny2d with fast e-ph (spectral radius ~0.27/fs) and slow ph-ph (~0.027/fs), from
    random populations so that every part is active."""
    wl = synth.build("tiny2d")
    P = dict(wl.problem_arrays())
    P["eph_g2"] = P["eph_g2"] * scale_eph
    P["pp_v2"] = P["pp_v2"] * scale_pp
    rng = np.random.default_rng(17)
    wl.y0 = np.concatenate([rng.uniform(0.05, 0.95, wl.n_el), rng.uniform(0.0, 2.0, wl.n_ph)])
    return wl, oracle.Oracle(P)


def test_rk4_and_mis_convergence_orders():
    wl, o = _coupled_problem()
    fast = lambda v: o.rhs(v, parts=3)
    slow = lambda v: o.rhs(v, parts=4)
    full = lambda v: o.rhs(v, parts=7)
    T = 40.0
    # reference: RK4 with a tiny step
    yref = wl.y0.copy()
    for _ in range(3200):
        yref = I.rk4_step(full, yref, T / 3200)
    errs_rk4, errs_mis = [], []
    for m in (8, 16, 32):
        h = T / m
        y = wl.y0.copy()
        for _ in range(m):
            y = I.rk4_step(full, y, h)
        errs_rk4.append(np.linalg.norm(y - yref))
        y = wl.y0.copy()
        solver = I.rk4_fixed_solver(h / 64)
        for _ in range(m):
            y = I.mis_step(fast, slow, y, h, solver)
        errs_mis.append(np.linalg.norm(y - yref))
    p_rk4 = np.log2(errs_rk4[1] / errs_rk4[2])
    p_mis = np.log2(errs_mis[1] / errs_mis[2])
    assert 3.6 < p_rk4 < 4.6, errs_rk4
    assert 2.6 < p_mis < 3.6, errs_mis


def test_embedded_order_three():
    wl, o = _coupled_problem()
    full = lambda v: o.rhs(v, parts=7)
    T = 40.0
    yref = wl.y0.copy()
    for _ in range(3200):
        yref = I.rk4_step(full, yref, T / 3200)
    errs = []
    for m in (32, 64, 128):
        y = wl.y0.copy()
        for _ in range(m):
            ynew, lte = I.erk_attempt(full, y, T / m)
            y = ynew - lte          # the embedded solution
        errs.append(np.linalg.norm(y - yref))
    p = np.log2(errs[1] / errs[2])
    assert 2.6 < p < 3.6, errs


def test_mis_reduces_to_base_erk_without_fast_part():
    wl, o = _coupled_problem()
    slow = lambda v: o.rhs(v, parts=4)
    zero = lambda v: np.zeros_like(v)
    h = 3.0
    y_mis = I.mis_step(zero, slow, wl.y0.copy(), h, I.rk4_fixed_solver(h / 7))
    kw = dict(I.KNOTH_WOLKE3)
    kw = dict(c=kw["c"], A=kw["A"], b=kw["b"], bt=kw["b"])
    y_erk, _ = I.erk_attempt(slow, wl.y0.copy(), h, tab=kw)
    assert np.allclose(y_mis, y_erk, rtol=0, atol=1e-15 * np.abs(wl.y0).max())


def test_mis_reduces_to_fast_integrator_without_slow_part():
    wl, o = _coupled_problem()
    fast = lambda v: o.rhs(v, parts=3)
    zero = lambda v: np.zeros_like(v)
    h = 3.0
    hf = 0.25
    y_mis = I.mis_step(fast, zero, wl.y0.copy(), h, I.rk4_fixed_solver(hf))
    # the same fast integrator over the three stage intervals
    y = wl.y0.copy()
    solver = I.rk4_fixed_solver(hf)
    for a, b in ((0.0, 1.0), (1.0, 2.25), (2.25, 3.0)):
        y = solver(y, a, b, fast)
    assert np.array_equal(y_mis, y)


def test_nonfinite_state_fails_the_step():
    wl = synth.build("toy2d")
    o = oracle.Oracle(wl.problem_arrays())
    y = wl.y0.copy(); y[3] = np.nan
    atol = np.full(wl.n_y, 1e-9)
    a = I.Adaptive(rhs=o.rhs, atol_vec=atol, c=I.Controls(), h=0.1)
    with pytest.raises(I.StepFailure):
        a.advance(y, 0.0, 1.0)


def test_too_many_failures_raise():
    wl = synth.build("toy2d")
    o = oracle.Oracle(wl.problem_arrays())
    atol = np.full(wl.n_y, 1e-30)
    a = I.Adaptive(rhs=o.rhs, atol_vec=atol, c=I.Controls(rtol=1e-15, max_fails=1), h=5.0)
    with pytest.raises(I.StepFailure):
        a.advance(wl.y0.copy(), 0.0, 10.0)


def test_split_step_special_cases():
    """Operator splitting: without a slow part it is the fast RK4 substeps;
    without a fast part it is one RK4 step of the slow part."""
    wl, o = _coupled_problem()
    fast = lambda v: o.rhs(v, parts=3)
    slow = lambda v: o.rhs(v, parts=4)
    zero = lambda v: np.zeros_like(v)
    hs, hf = 3.0, 0.7
    y = I.split_step(fast, zero, wl.y0.copy(), hs, hf)
    v = wl.y0.copy()
    for h in (0.7, 0.7, 0.7, 0.7, 0.2):
        v = I.rk4_step(fast, v, h)
    assert np.allclose(y, v, rtol=0, atol=1e-15)
    y = I.split_step(zero, slow, wl.y0.copy(), hs, hf)
    assert np.array_equal(y, I.rk4_step(slow, wl.y0.copy(), hs))


def test_split_step_is_first_order():
    """Lie splitting of coupled parts converges at first order in h_s (fast
    substeps small enough that RK4's own error does not show)."""
    wl, o = _coupled_problem()
    fast = lambda v: o.rhs(v, parts=3)
    slow = lambda v: o.rhs(v, parts=4)
    full = lambda v: o.rhs(v, parts=7)
    T = 40.0
    yref = wl.y0.copy()
    for _ in range(3200):
        yref = I.rk4_step(full, yref, T / 3200)
    errs = []
    for m in (8, 16, 32):
        y = wl.y0.copy()
        for _ in range(m):
            y = I.split_step(fast, slow, y, T / m, T / m / 32)
        errs.append(np.linalg.norm(y - yref))
    p = np.log2(errs[1] / errs[2])
    assert 0.8 < p < 1.3, errs


def _linear_fast_slow(n=6, seed=3):
    """y' = A_f y + A_s y with non-commuting symmetric negative definite
    parts (fast eigenvalues -1 .. -2, slow -0.05 .. -0.2) and the exact fast
    flow of v' = A_f v + r (r constant): v(t) = e^{A_f t} v0 + A_f^{-1}(e^{A_f t} - I) r."""
    from scipy.linalg import expm
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
    Af = Q1 @ np.diag(-np.linspace(1.0, 2.0, n)) @ Q1.T
    As = Q2 @ np.diag(-np.linspace(0.05, 0.2, n)) @ Q2.T
    Afi = np.linalg.inv(Af)

    def exact_fast(v, t0, t1, f):
        r = f(np.zeros(n))            # the constant forcing of the stage
        E = expm(Af * (t1 - t0))
        return E @ v + Afi @ ((E - np.eye(n)) @ r)

    y0 = rng.uniform(0.5, 1.5, n)
    return Af, As, exact_fast, y0, (lambda H, y: expm((Af + As) * H) @ y)


def test_step_doubling_estimate_is_the_local_error():
    """(y_half - y_full)/7 approaches exact - y_half as H -> 0 (MIS order 3
    with an exact fast flow), and shrinks like H^4."""
    Af, As, fsolve, y0, flow = _linear_fast_slow()
    M = I.MisAdaptive(lambda v: Af @ v, lambda v: As @ v, fsolve, np.full(len(y0), 1e-12),
                      I.Controls(rtol=1.0, atol_el=1e-12, atol_ph=1e-12))
    sizes, ratios = [], []
    for H in (0.4, 0.2, 0.1, 0.05):
        yf = I.mis_step(M.fast_rhs, M.slow_rhs, y0, H, fsolve)
        yh = I.mis_step(M.fast_rhs, M.slow_rhs, y0, H / 2, fsolve)
        yh = I.mis_step(M.fast_rhs, M.slow_rhs, yh, H / 2, fsolve)
        est = (yh - yf) / 7.0
        true = flow(H, y0) - yh
        sizes.append(np.linalg.norm(est))
        ratios.append(np.linalg.norm(est - true) / np.linalg.norm(true))
        # the oracle's attempt computes the same estimate
        yh2, eps = M.attempt(y0, H)
        assert np.array_equal(yh2, yh)
        assert abs(eps - I.wrms(est, y0, 1.0, np.full(len(y0), 1e-12))) <= 1e-15 * eps
    assert ratios[-1] < 0.05 and ratios[-1] < ratios[0]
    for a, b in zip(sizes, sizes[1:]):
        assert 12.0 < a / b < 20.0


def test_adaptive_slow_step_meets_tolerance():
    """Global error at t_end falls with the tolerance (error-per-step control
    of a third-order method: about tol^(3/4), 30x per 100x), stays within a
    modest multiple of it, and the run lands on t_end; a too-large first
    step is rejected and recovered from."""
    Af, As, fsolve, y0, flow = _linear_fast_slow()
    T = 4.0   # the solution decays by e^-4: relative errors stay meaningful
    exact = flow(T, y0)
    errs = []
    for rtol in (1e-4, 1e-6, 1e-8):
        atol = np.full(len(y0), rtol * 1e-3)
        M = I.MisAdaptive(lambda v: Af @ v, lambda v: As @ v, fsolve, atol,
                          I.Controls(rtol=rtol, atol_el=rtol * 1e-3, atol_ph=rtol * 1e-3), H=0.5)
        y, t = M.advance(y0.copy(), 0.0, T)
        assert t == T and M.history[-1][0] == T
        errs.append(np.linalg.norm(y - exact) / np.linalg.norm(exact))
        assert errs[-1] <= 30 * rtol
    assert errs[0] > 10 * errs[1] > 100 * errs[2]
    M = I.MisAdaptive(lambda v: Af @ v, lambda v: As @ v, fsolve, np.full(len(y0), 1e-10),
                      I.Controls(rtol=1e-7, atol_el=1e-10, atol_ph=1e-10), H=25.0)
    y, t = M.advance(y0.copy(), 0.0, T)
    assert M.n_reject >= 1 and t == T
    assert np.linalg.norm(y - exact) / np.linalg.norm(exact) <= 30e-7


def test_slow_controller_is_an_i_controller():
    """eta = safety eps^(-1/4) whatever the history; limits as for the ERK."""
    c = I.slow_controls(I.Controls())
    for eps in (1e-3, 0.5, 0.9):
        for e1, e2 in ((1.0, 1.0), (0.2, 3.0)):
            assert abs(I.pid_eta(eps, e1, e2, True, False, c) - min(c.safety * eps ** -0.25, c.eta_max)) < 1e-15
    assert I.pid_eta(50.0, 1.0, 1.0, False, False, c) == max(c.safety * 50.0 ** -0.25, c.eta_fail_min)


def _stack_linear(systems):
    """Independent linear fast/slow systems stacked in one vector: block
    diagonal operators, the slices, and a per-slice exact fast solver."""
    from scipy.linalg import block_diag
    Afb = block_diag(*[s[0] for s in systems])
    Asb = block_diag(*[s[1] for s in systems])
    sizes = [len(s[3]) for s in systems]
    offs = np.cumsum([0] + sizes)
    slices = [slice(int(a), int(b)) for a, b in zip(offs[:-1], offs[1:])]
    solver = I.SliceFastSolver(slices, [s[2] for s in systems])
    return Afb, Asb, slices, solver, np.concatenate([s[3] for s in systems])


def test_batched_slow_step_meets_each_instance_tolerance():
    """Two different instances sharing the slow step: the step passes only if
    both pass, so each instance ends within the tolerance-sized distance of
    its own exact solution, and the common clock lands on t_end."""
    A, B = _linear_fast_slow(seed=1), _linear_fast_slow(seed=2)
    Afb, Asb, slices, solver, y0 = _stack_linear([A, B])
    T, rtol = 4.0, 1e-6
    atol = np.full(len(y0), rtol * 1e-3)
    M = I.MisAdaptive(lambda v: Afb @ v, lambda v: Asb @ v, solver, atol,
                      I.Controls(rtol=rtol, atol_el=rtol * 1e-3, atol_ph=rtol * 1e-3), H=0.5,
                      norm=I.batch_norm(slices, rtol, atol))
    y, t = M.advance(y0.copy(), 0.0, T)
    assert t == T and M.n_accept >= 5
    for s, sys_ in zip(slices, (A, B)):
        exact = sys_[4](T, sys_[3])
        assert np.linalg.norm(y[s] - exact) / np.linalg.norm(exact) <= 30 * rtol
    # the norm is the largest instance norm
    est = np.random.default_rng(0).standard_normal(len(y0)) * 1e-6
    per = [I.wrms(est[s], y0[s], rtol, atol[s]) for s in slices]
    assert I.batch_norm(slices, rtol, atol)(est, y0) == max(per) and per[0] != per[1]


def test_batched_slow_step_with_a_quiet_instance_is_the_instance_alone():
    """An instance whose state never moves (zero solution) has a zero error
    estimate, so a batch of it with A takes A's accepted and rejected steps,
    and A's slice ends where A alone ends."""
    n = 6
    A = _linear_fast_slow(seed=3, n=n)
    Z = (-np.eye(n), np.zeros((n, n)), None, np.zeros(n), None)
    Zf = -np.eye(n)

    def z_fast(v, t0, t1, f):
        return np.exp(-(t1 - t0)) * v + (1.0 - np.exp(-(t1 - t0))) * f(np.zeros(n))   # exact for v' = -v + r

    Afb, Asb, slices, solver, y0 = _stack_linear([A, (Zf, Z[1], z_fast, Z[3])])
    rtol = 1e-6
    atol = np.full(len(y0), 1e-9)
    Mb = I.MisAdaptive(lambda v: Afb @ v, lambda v: Asb @ v, solver, atol,
                       I.Controls(rtol=rtol, atol_el=1e-9, atol_ph=1e-9), H=0.5,
                       norm=I.batch_norm(slices, rtol, atol))
    yb, tb = Mb.advance(y0.copy(), 0.0, 3.0)
    Ma = I.MisAdaptive(lambda v: A[0] @ v, lambda v: A[1] @ v, A[2], atol[:n],
                       I.Controls(rtol=rtol, atol_el=1e-9, atol_ph=1e-9), H=0.5)
    ya, ta = Ma.advance(A[3].copy(), 0.0, 3.0)
    assert tb == ta == 3.0 and (Mb.n_accept, Mb.n_reject) == (Ma.n_accept, Ma.n_reject)
    # the same steps up to rounding (the estimate is a difference of nearly
    # equal states, so rounding of the stacked products moves H at ~1e-11)
    assert np.allclose([h[1] for h in Mb.history], [h[1] for h in Ma.history], rtol=1e-8, atol=0)
    assert np.allclose(yb[slices[0]], ya, rtol=1e-10, atol=1e-15)
    assert np.all(yb[slices[1]] == 0.0)


@pytest.mark.parametrize("case", ["tiny2d", "linear", "quiet", "small_state"])
def test_starting_step_matches_scipy(case):
    """The Hairer-Norsett-Wanner starting step (Solving ODEs I, II.4) against
    SciPy's own implementation of the same algorithm (select_initial_step,
    RMS norm with scale atol + rtol |y0|, no interval or step cap), in each
    of its branches: a nonlinear collision right-hand side, a linear system,
    a right-hand side that vanishes (d1 = d2 = 0) and a tiny state
    (d0 < 1e-5)."""
    from scipy.integrate._ivp.common import select_initial_step
    import oracle
    import synth
    c = I.Controls(rtol=1e-6, atol_el=1e-9, atol_ph=1e-12)
    if case == "tiny2d":
        wl = synth.build("tiny2d")
        o = oracle.Oracle(wl.problem_arrays())
        rhs, y0 = (lambda v: o.rhs(v)), wl.y0.copy()
        atol = np.concatenate([np.full(wl.n_el, c.atol_el), np.full(wl.n_ph, c.atol_ph)])
    else:
        rng = np.random.default_rng(4)
        A = -np.diag(rng.uniform(0.1, 3.0, 8))
        rhs = (lambda v: np.zeros_like(v)) if case == "quiet" else (lambda v: A @ v)
        y0 = rng.uniform(0.5, 1.5, 8) * (1e-12 if case == "small_state" else 1.0)
        atol = np.full(8, c.atol_el)
    h = I.hnw_initial_step(rhs, y0, c, atol, order=4)
    ref = select_initial_step(lambda t, v: rhs(v), 0.0, y0, 1e300, np.inf, rhs(y0), 1.0, 4, c.rtol, atol)
    assert abs(h - ref) <= 1e-13 * ref, (h, ref)
