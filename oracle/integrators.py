"""Oracle time integrators for y' = f(t, y) (Eq. (erk_ode)) and the split
y' = f^f + f^s (Eq. (mri_ode)).  TEST INFRASTRUCTURE ONLY (see package doc).

Plain numpy, FP64, one vector operation per formula term:

* ``rk4_step``           classical fixed-step RK4 (the prior-work baseline);
* ``erk_attempt``        one attempted step of an explicit RK pair, Eq. (ERK_method),
                         with the Zonneveld 5-stage 4(3) tableau;
* ``wrms``               Eq. (wrms_norm) with weights Eq. (wrms_weights);
* ``pid_eta``            Eq. (pid_controller) plus the safeguards read in for it;
* ``Adaptive``           the accept/reject loop of the ERK method;
* ``mis_step``           one slow step of the MRI algorithm with the MIS coupling
                         Eq. (mis_coef) built from the Knoth-Wolke 3-stage ERK.
* ``MisAdaptive``        MIS with the slow step chosen by step doubling (the
                         slow-step adaptivity the Discussion leaves open);
                         ``batch_norm`` and ``SliceFastSolver`` run it on stacked
                         independent instances that share the slow step.

``hnw_initial_step`` (the starting-step heuristic of Hairer, Norsett and
Wanner, not from the paper) is pinned against SciPy's implementation of the
same algorithm in each of its branches.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction as Fr

import numpy as np

# ----------------------------------------------------------------- tableaux
# Zonneveld 5-stage pair, main order 4, embedding order 3 (Methods, ERK method:
# the default ARKODE ERK).  Its main weights coincide with classical RK4.
ZONNEVELD = dict(
    c=[Fr(0), Fr(1, 2), Fr(1, 2), Fr(1), Fr(3, 4)],
    A=[[],
       [Fr(1, 2)],
       [Fr(0), Fr(1, 2)],
       [Fr(0), Fr(0), Fr(1)],
       [Fr(5, 32), Fr(7, 32), Fr(13, 32), Fr(-1, 32)]],
    b=[Fr(1, 6), Fr(1, 3), Fr(1, 3), Fr(1, 6), Fr(0)],
    bt=[Fr(-1, 2), Fr(7, 3), Fr(7, 3), Fr(13, 6), Fr(-16, 3)],
    order=4, emb_order=3,
)

# Classical RK4.
RK4 = dict(
    c=[Fr(0), Fr(1, 2), Fr(1, 2), Fr(1)],
    A=[[], [Fr(1, 2)], [Fr(0), Fr(1, 2)], [Fr(0), Fr(0), Fr(1)]],
    b=[Fr(1, 6), Fr(1, 3), Fr(1, 3), Fr(1, 6)],
)

# Knoth-Wolke 3-stage, 3rd-order ERK: the base method of the MIS scheme
# (Methods, MRI method).
KNOTH_WOLKE3 = dict(
    c=[Fr(0), Fr(1, 3), Fr(3, 4)],
    A=[[], [Fr(1, 3)], [Fr(-3, 16), Fr(15, 16)]],
    b=[Fr(1, 6), Fr(3, 10), Fr(8, 15)],
)


def mis_coupling(base: dict):
    """MIS abscissae c_hat = [c_1..c_S, 1] and coupling Omega (K = 1) of
    Eq. (mis_coef).  The last row is taken as b_j - A_{S,j}: with it the stage
    increments telescope to the base method's b (the printed A_{S-1,j} would
    not even give a consistent method)."""
    S = len(base["b"])
    A = [list(row) + [Fr(0)] * (S - len(row)) for row in base["A"]]
    chat = list(base["c"]) + [Fr(1)]
    Om = [[Fr(0)] * S for _ in range(S + 1)]
    for i in range(1, S):          # 2 <= i <= S (1-based): A_i - A_{i-1}
        Om[i] = [A[i][j] - A[i - 1][j] for j in range(S)]
    Om[S] = [base["b"][j] - A[S - 1][j] for j in range(S)]  # i = S+1 = S_hat
    return chat, Om


def _f(x):
    return float(x)


# ---------------------------------------------------------------- RK kernels
def rk4_step(rhs, y, h):
    """One classical RK4 step (fixed step size h)."""
    k1 = rhs(y)
    k2 = rhs(y + (h * 0.5) * k1)
    k3 = rhs(y + (h * 0.5) * k2)
    k4 = rhs(y + h * k3)
    return y + h * (k1 / 6.0 + k2 / 3.0 + k3 / 3.0 + k4 / 6.0)


def erk_attempt(rhs, y, h, tab=ZONNEVELD):
    """Stages z_i = y + h sum_{j<i} A_ij f(z_j); solution y + h sum b_i k_i and
    local error estimate LTE = y_k - ytilde_k = h sum (b_i - btilde_i) k_i."""
    ks = []
    for i in range(len(tab["b"])):
        z = y.copy()
        for j, a in enumerate(tab["A"][i]):
            if a != 0:
                z += (h * _f(a)) * ks[j]
        ks.append(rhs(z))
    ynew = y.copy()
    lte = np.zeros_like(y)
    for i, k in enumerate(ks):
        if tab["b"][i] != 0:
            ynew += (h * _f(tab["b"][i])) * k
        d = tab["b"][i] - tab["bt"][i]
        if d != 0:
            lte += (h * _f(d)) * k
    return ynew, lte


def wrms(v, y_prev, rtol, atol_vec):
    """||v||_WRMS with w_i = 1/(rtol |y_prev,i| + atol_i)."""
    w = 1.0 / (rtol * np.abs(y_prev) + atol_vec)
    return float(np.sqrt(np.mean((v * w) ** 2)))


# ----------------------------------------------------------------- control
@dataclass
class Controls:
    rtol: float = 1e-6
    atol_el: float = 1e-9
    atol_ph: float = 1e-12
    # PID gains and order (Methods, Eq. (pid_controller))
    k1: float = 0.58
    k2: float = 0.21
    k3: float = 0.10
    order: int = 4
    alt_sign: bool = False     # True: +k2 on eps_{k-1} (Soderlind PID form)
    # safeguards (not given by the paper)
    safety: float = 0.96
    eta_max: float = 20.0
    eta_max_first: float = 1e4
    eta_fail_min: float = 0.1
    eta_fail_max: float = 0.9
    # from the small_nef-th consecutive error-test failure on, the ratio is
    # also capped by eta_fail_repeat (a rescue for steps that the history
    # factors keep from shrinking; the paper prints no safeguards)
    small_nef: int = 5
    eta_fail_repeat: float = 0.3
    eps_floor: float = 1e-10
    max_fails: int = 7


def pid_eta(eps, e1, e2, accepted: bool, first: bool, c: Controls, fails: int = 1) -> float:
    """Step ratio h'/h: safety * eps_k^(-k1/p) eps_{k-1}^(-+k2/p) eps_{k-2}^(-k3/p),
    then limited to [.., eta_max] on acceptance or [eta_fail_min, eta_fail_max]
    on rejection, and to <= eta_fail_repeat once `fails` (consecutive
    failures, this one included) reaches small_nef."""
    e0 = max(eps, c.eps_floor)
    s2 = 1.0 if c.alt_sign else -1.0
    eta = (c.safety * e0 ** (-c.k1 / c.order) * max(e1, c.eps_floor) ** (s2 * c.k2 / c.order)
           * max(e2, c.eps_floor) ** (-c.k3 / c.order))
    if accepted:
        return min(eta, c.eta_max_first if first else c.eta_max)
    eta = min(max(eta, c.eta_fail_min), c.eta_fail_max)
    return min(eta, c.eta_fail_repeat) if fails >= c.small_nef else eta


def hnw_initial_step(rhs, y0, c: Controls, atol_vec, order=4):
    """Starting step size of Hairer, Norsett & Wanner (Solving ODEs I, II.4),
    measured in the WRMS norm of the current tolerances."""
    f0 = rhs(y0)
    d0 = wrms(y0, y0, c.rtol, atol_vec)
    d1 = wrms(f0, y0, c.rtol, atol_vec)
    h0 = 0.01 * d0 / d1 if (d0 >= 1e-5 and d1 >= 1e-5) else 1e-6
    y1 = y0 + h0 * f0
    d2 = wrms(rhs(y1) - f0, y0, c.rtol, atol_vec) / h0
    m = max(d1, d2)
    h1 = (0.01 / m) ** (1.0 / (order + 1)) if m > 1e-15 else max(1e-6, h0 * 1e-3)
    return min(100.0 * h0, h1)


class StepFailure(RuntimeError):
    pass


@dataclass
class Adaptive:
    """Adaptive Zonneveld ERK on y' = rhs(y), with the WRMS test ||LTE|| <= 1
    (Methods, ERK method).  The error history starts at 1 and is updated on
    accepted steps only."""
    rhs: object
    atol_vec: np.ndarray
    c: Controls = field(default_factory=Controls)
    h: float = 0.0
    e1: float = 1.0
    e2: float = 1.0
    first: bool = True
    n_accept: int = 0
    n_reject: int = 0
    n_rhs: int = 0
    history: list = field(default_factory=list)   # (t_new, h_used, eps) of accepted steps

    def _rhs(self, y):
        self.n_rhs += 1
        return self.rhs(y)

    def attempt(self, y, h):
        """One attempted step: returns (y_new, eps)."""
        ynew, lte = erk_attempt(self._rhs, y, h)
        return ynew, wrms(lte, y, self.c.rtol, self.atol_vec)

    def advance(self, y, t, t_out, one_step=False, h_max=None):
        """Advance from t toward t_out; returns (y, t).  The last step is cut to
        land on t_out."""
        if self.h <= 0.0:
            self.h = hnw_initial_step(self._rhs, y, self.c, self.atol_vec)
        fails = 0
        while t < t_out:
            h = self.h if h_max is None else min(self.h, h_max)
            last = t + h >= t_out
            if last:
                h = t_out - t
            ynew, eps = self.attempt(y, h)
            if not np.isfinite(eps):
                raise StepFailure("non-finite error estimate")
            if eps <= 1.0:
                self.h = h * pid_eta(eps, self.e1, self.e2, True, self.first, self.c)
                self.e2, self.e1 = self.e1, max(eps, self.c.eps_floor)
                self.first = False
                y = ynew
                t = t_out if last else t + h
                self.n_accept += 1
                self.history.append((t, h, eps))
                fails = 0
                if one_step:
                    break
            else:
                fails += 1
                self.h = h * pid_eta(eps, self.e1, self.e2, False, self.first, self.c, fails)
                self.n_reject += 1
                if fails > self.c.max_fails:
                    raise StepFailure("too many consecutive error-test failures")
        return y, t


def replay(rhs, y, steps):
    """Re-run a recorded sequence of accepted step sizes with the Zonneveld
    main solution (the same arithmetic as an accepted adaptive step)."""
    for h in steps:
        y, _ = erk_attempt(rhs, y, h)
    return y


# --------------------------------------------------------------------- MIS
def mis_step(fast_rhs, slow_rhs, y, h_s, fast_solve, base=KNOTH_WOLKE3):
    """One slow step of the MRI algorithm (Methods, MRI method) with MIS
    coupling: z_1 = y; for i = 2..S_hat solve v' = f^f(v) + r_i on
    [c_{i-1} h_s, c_i h_s] from z_{i-1} with the constant forcing
    r_i = (1/dc_i) sum_{j<i} Omega_ij f^s(z_j); y_new = z_{S_hat}.

    fast_solve(v0, t0, t1, forced_rhs) -> v(t1) integrates the fast problem."""
    chat, Om = mis_coupling(base)
    z = [y]
    fs = [slow_rhs(y)]
    for i in range(1, len(chat)):
        dc = chat[i] - chat[i - 1]
        r = np.zeros_like(y)
        for j in range(i):
            if Om[i][j] != 0:
                r += _f(Om[i][j] / dc) * fs[j]

        def forced(v, r=r):
            return fast_rhs(v) + r

        v = fast_solve(z[i - 1], _f(chat[i - 1]) * h_s, _f(chat[i]) * h_s, forced)
        z.append(v)
        if i < len(chat) - 1:
            fs.append(slow_rhs(v))
    return z[-1]


def rk4_fixed_solver(h_fast):
    """Fast solver: classical RK4 with step h_fast, last substep cut to land."""
    def solve(v, t0, t1, f):
        t = t0
        while t < t1:
            h = min(h_fast, t1 - t)
            last = t + h_fast >= t1
            if last:
                h = t1 - t
            v = rk4_step(f, v, h)
            t = t1 if last else t + h
        return v
    return solve


def split_step(fast_rhs, slow_rhs, y, h_s, h_f):
    """One step of the first-order operator splitting the paper compares
    against (Results, discussion of Fig. 3): the fast part advanced over
    [t, t + h_s] by RK4 with steps h_f (the last cut to land), then the slow
    part advanced over the same interval by one RK4 step of h_s."""
    y = rk4_fixed_solver(h_f)(y, 0.0, h_s, fast_rhs)
    return rk4_step(slow_rhs, y, h_s)


class AdaptiveFastSolver:
    """Fast solver: adaptive Zonneveld ERK whose step size and error history
    carry over from one stage interval to the next, capped by the interval."""

    def __init__(self, atol_vec, c: Controls, h0: float):
        self.atol_vec = atol_vec
        self.c = c
        self.h = h0
        self.e1 = 1.0
        self.e2 = 1.0
        self.first = True
        self.n_accept = 0
        self.n_reject = 0

    def __call__(self, v, t0, t1, f):
        a = Adaptive(rhs=f, atol_vec=self.atol_vec, c=self.c, h=self.h, e1=self.e1,
                     e2=self.e2, first=self.first)
        v, _ = a.advance(v, t0, t1, h_max=t1 - t0)
        self.h, self.e1, self.e2, self.first = a.h, a.e1, a.e2, a.first
        self.n_accept += a.n_accept
        self.n_reject += a.n_reject
        return v


# ------------------------------------------------------- adaptive slow step
def slow_controls(c: Controls) -> Controls:
    """Controller of the slow step: an I controller on the step-doubling
    estimate of a third-order method, eta = safety * eps^(-1/4), with the
    safeguards of c (the paper leaves slow-step adaptivity to future work;
    this is the textbook choice for a method without an embedded pair)."""
    return Controls(rtol=c.rtol, atol_el=c.atol_el, atol_ph=c.atol_ph, k1=1.0, k2=0.0, k3=0.0, order=4,
                    alt_sign=False, safety=c.safety, eta_max=c.eta_max, eta_max_first=c.eta_max_first,
                    eta_fail_min=c.eta_fail_min, eta_fail_max=c.eta_fail_max, eps_floor=c.eps_floor,
                    max_fails=c.max_fails, small_nef=c.small_nef, eta_fail_repeat=c.eta_fail_repeat)


@dataclass
class MisAdaptive:
    """MRI (MIS) with the slow step chosen by step doubling (Hairer, Norsett &
    Wanner, Solving ODEs I, II.4): an attempt of size H takes one MIS step of
    H and two of H/2 from the same state; the two-half-step result is kept
    and its local error is estimated by (y_half - y_full) / (2^3 - 1), the
    MIS order being 3.  The estimate's WRMS norm (weights from the state at
    the start of the attempt) decides acceptance; the step ratio comes from
    slow_controls.  The fast solver is called in the order full step, first
    half, second half, and keeps its own state across attempts."""
    fast_rhs: object
    slow_rhs: object
    fast_solve: object
    atol_vec: np.ndarray
    c: Controls = field(default_factory=Controls)
    H: float = 1.0
    e1: float = 1.0
    e2: float = 1.0
    first: bool = True
    n_accept: int = 0
    n_reject: int = 0
    history: list = field(default_factory=list)   # (t_new, H_used, eps) of accepted steps
    norm: object = None    # norm(est, y) -> eps; None: the WRMS norm over the whole vector

    def attempt(self, y, H):
        """(y_half, eps) of one attempt of size H from y."""
        y_full = mis_step(self.fast_rhs, self.slow_rhs, y, H, self.fast_solve)
        y_half = mis_step(self.fast_rhs, self.slow_rhs, y, H / 2, self.fast_solve)
        y_half = mis_step(self.fast_rhs, self.slow_rhs, y_half, H / 2, self.fast_solve)
        est = (y_half - y_full) / 7.0
        if self.norm is not None:
            return y_half, self.norm(est, y)
        return y_half, wrms(est, y, self.c.rtol, self.atol_vec)

    def advance(self, y, t, t_out, one_step=False):
        cs = slow_controls(self.c)
        fails = 0
        while t < t_out:
            H = self.H
            last = t + H >= t_out
            if last:
                H = t_out - t
            ynew, eps = self.attempt(y, H)
            if not np.isfinite(eps):
                raise StepFailure("non-finite error estimate")
            if eps <= 1.0:
                self.H = H * pid_eta(eps, self.e1, self.e2, True, self.first, cs)
                self.e2, self.e1 = self.e1, max(eps, cs.eps_floor)
                self.first = False
                y = ynew
                t = t_out if last else t + H
                self.n_accept += 1
                self.history.append((t, H, eps))
                fails = 0
                if one_step:
                    break
            else:
                fails += 1
                self.H = H * pid_eta(eps, self.e1, self.e2, False, self.first, cs, fails)
                self.n_reject += 1
                if fails > cs.max_fails:
                    raise StepFailure("too many consecutive error-test failures")
        return y, t


# ------------------------------------------- batches with a common slow step
def batch_norm(slices, rtol, atol_vec):
    """Error norm of independent instances stacked in one vector that share
    the slow step: the step passes only if every instance passes its own WRMS
    test, so the norm is the largest instance norm (each with its own
    weights)."""
    def norm(est, y):
        return max(wrms(est[s], y[s], rtol, atol_vec[s]) for s in slices)
    return norm


class SliceFastSolver:
    """Fast solver of stacked independent instances: each slice integrated by
    its own solver (own step size and error history).  The forced right-hand
    side f of the stacked vector is separable, so a slice's right-hand side is
    f evaluated with the other slices held at their starting values."""

    def __init__(self, slices, solvers):
        self.slices = list(slices)
        self.solvers = list(solvers)

    def __call__(self, v, t0, t1, f):
        out = v.copy()
        for s, solve in zip(self.slices, self.solvers):
            def f_s(u, s=s):
                w = v.copy()
                w[s] = u
                return f(w)[s]
            out[s] = solve(v[s].copy(), t0, t1, f_s)
        return out
