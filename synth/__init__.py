"""Seeded synthetic inputs for the coupled electron-phonon rt-BTE.

This package builds the *inputs* of the collision-integral problem (grid,
band energies, phonon energies, stored e-ph / ph-ph channels with their
|g|^2 and |V3|^2 values, initial populations).  It contains none of the
method's arithmetic (no delta weights, no truncation, no occupation factors,
no sums), so it can feed both the CPU oracle and the GPU library without
coupling them.  The heavy enumeration lives in ``gen.cpp`` (C++/OpenMP,
Philox4x32-10 counter-based randomness); this module wraps it with ctypes and
holds the named workload recipes.

The paper's first-principles graphene and silicon matrices (Methods,
grid-size paragraphs) are not available, so these recipes stand in for them
with the same grid sizes, band/branch counts, Gaussian widths and cutoffs.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HBAR_EV_FS = 0.6582119569      # reduced Planck constant, eV*fs (CODATA 2018, exact)
KB_EV_PER_K = 8.617333262e-5   # Boltzmann constant, eV/K (CODATA 2018, exact)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


# RTBTE_HOST_SANITIZE=1 selects a build of the same source under
# AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the
# process must preload the sanitizer runtimes).
_SANITIZE = os.environ.get("RTBTE_HOST_SANITIZE") == "1"
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer", "-g"]


def lib_path(sanitized=None) -> str:
    san = _SANITIZE if sanitized is None else sanitized
    return os.path.join(_HERE, "libsynth_san.so" if san else "libsynth.so")


def build_lib(sanitized=None) -> str:
    """Compile gen.cpp into libsynth.so (host g++, OpenMP); with sanitized
    (default: RTBTE_HOST_SANITIZE) into libsynth_san.so under ASan and UBSan."""
    import subprocess
    san = _SANITIZE if sanitized is None else sanitized
    out = lib_path(san)
    cmd = (["g++", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-Wall"] +
           (SANITIZE_FLAGS if san else []) + ["-o", out + ".tmp", os.path.join(_HERE, "gen.cpp")])
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            raise RuntimeError("synth/libsynth.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(lib_path())
        L.synth_create.restype = ctypes.c_void_p
        L.synth_create.argtypes = [ctypes.POINTER(Params)]
        L.synth_destroy.argtypes = [ctypes.c_void_p]
        L.synth_sizes.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.synth_states.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        L.synth_fill_eph.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.synth_fill_pp.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 4
        L.synth_dense.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.synth_philox4x32_10.argtypes = [ctypes.c_void_p] * 3
        L.synth_threads.restype = ctypes.c_int
        L.synth_set_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("lattice", ctypes.c_int32),
        ("n_bands", ctypes.c_int32), ("n_modes", ctypes.c_int32),
        ("with_eph", ctypes.c_int32), ("with_pp", ctypes.c_int32),
        ("quantize", ctypes.c_int32), ("quantum", ctypes.c_double),
        ("t_hop", ctypes.c_double), ("win_lo", ctypes.c_double), ("win_hi", ctypes.c_double),
        ("shell_eph", ctypes.c_double), ("shell_pp", ctypes.c_double),
        ("keep_eph", ctypes.c_double), ("keep_pp", ctypes.c_double),
        ("g2_mu", ctypes.c_double), ("g2_sig", ctypes.c_double),
        ("v2_mu", ctypes.c_double), ("v2_sig", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("keep_pp_q", ctypes.c_double),
    ]


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def philox4x32_10(ctr, key):
    """Philox4x32-10 block function (for known-answer tests)."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _lib().synth_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def set_threads(n: int) -> None:
    """OpenMP threads used by the enumeration (results do not depend on it)."""
    _lib().synth_set_threads(int(n))


def fermi_dirac(eps, T, mu=0.0):
    """Fermi-Dirac occupation at temperature T (K) and chemical potential mu (eV)."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / (KB_EV_PER_K * T)
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def solve_mu(eps, T, density, n_k_total):
    """Chemical potential (eV) at which the windowed states hold `density`
    carriers per cell at temperature T (bisection; the count rises with mu)."""
    lo, hi = float(np.min(eps)) - 5.0, float(np.max(eps)) + 5.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fermi_dirac(eps, T, mid).sum() / n_k_total < density:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def bose_einstein(hw, T):
    """Bose-Einstein occupation of phonons of energy hw (eV); 0 where hw <= 0."""
    hw = np.asarray(hw, dtype=np.float64)
    out = np.zeros_like(hw)
    pos = hw > 0
    out[pos] = 1.0 / np.expm1(hw[pos] / (KB_EV_PER_K * T))
    return out


MASTER_SEED = 2412134020
STREAM_PP = 0x70707033   # fourth Philox counter word of the |V3|^2 draws (gen.cpp)

# Workload recipes.  Each recipe fixes the model, the problem parameters that
# the method takes (sigma, n_sigma, hw_cut) and the initial state.
RECIPES = {
    # 18x18 square-lattice toy, e-ph only (2 cos tight-binding bands, 3 modes).
    "toy2d": dict(
        grid=dict(dim=2, L=18, lattice=0, n_bands=2, n_modes=3, t_hop=1.0,
                  win_lo=-0.5, win_hi=0.5, with_eph=1, with_pp=0,
                  shell_eph=0.075, shell_pp=0.0, keep_eph=1.0, keep_pp=0.0,
                  g2_mu=-3.0, g2_sig=1.0, v2_mu=0.0, v2_sig=1.0),
        problem=dict(sigma_eph=0.010, sigma_pp=0.002, nsigma=6.0, hw_cut=0.001),
        init=dict(T_el=2000.0, T_ph=300.0, mu=0.0),
        seed_offset=1,
    ),
    # Graphene-like coupled workload: 120x120 triangular k = q grid, two
    # nearest-neighbour pi bands (t = 3.09 eV, v = 1e6 m/s at K), six branches
    # in 0-200 meV, sigma 20 meV (e-ph) / 2 meV (ph-ph), 1 meV cutoff (Methods,
    # graphene grids).  The full pi bands are kept (~1.6e8 electron-side and
    # ~0.8e8 phonon-side e-ph channels); ph-ph triplets are thinned to ~5e8
    # channels (~7.8e8 stored entries: a third of the orderings of a triplet
    # conserve energy in neither of their two processes).  |g|^2 is scaled so that the e-ph Jacobian's spectral radius is
    # ~0.5/fs (explicit steps of a few fs), |V3|^2 so that the mean 300 K
    # phonon decay rate is ~1/ps.  Carriers start hot (4000 K), phonons at 300 K.
    "graphene2d": dict(
        grid=dict(dim=2, L=120, lattice=1, n_bands=2, n_modes=6, t_hop=3.09,
                  win_lo=-10.0, win_hi=10.0, with_eph=1, with_pp=1,
                  shell_eph=0.13, shell_pp=0.013, keep_eph=1.0, keep_pp=0.115,
                  g2_mu=-6.5, g2_sig=1.0, v2_mu=-16.33, v2_sig=1.0),
        problem=dict(sigma_eph=0.020, sigma_pp=0.002, nsigma=6.0, hw_cut=0.001),
        init=dict(T_el=4000.0, T_ph=300.0, mu=0.0),
        seed_offset=2,
    ),
    # Tiny coupled graphene-like grid (brute-force comparisons): wide Gaussians
    # so that a 6x6 grid still has channels of every kind.
    "tiny2d": dict(
        grid=dict(dim=2, L=6, lattice=1, n_bands=2, n_modes=6, t_hop=3.09,
                  win_lo=-10.0, win_hi=10.0, with_eph=1, with_pp=1,
                  shell_eph=0.45, shell_pp=0.045, keep_eph=1.0, keep_pp=1.0,
                  g2_mu=-4.0, g2_sig=1.0, v2_mu=-10.0, v2_sig=1.0),
        problem=dict(sigma_eph=0.08, sigma_pp=0.008, nsigma=5.0, hw_cut=0.001),
        init=dict(T_el=4000.0, T_ph=300.0, mu=0.0),
        seed_offset=11,
    ),
    # Tiny silicon-like 3D grid (3x3x3, 4 conduction bands, 6 branches).
    "tiny3d": dict(
        grid=dict(dim=3, L=3, lattice=2, n_bands=4, n_modes=6, t_hop=0.5,
                  win_lo=-1.0, win_hi=10.0, with_eph=1, with_pp=1,
                  shell_eph=0.35, shell_pp=0.035, keep_eph=1.0, keep_pp=1.0,
                  g2_mu=-4.0, g2_sig=1.0, v2_mu=-10.0, v2_sig=1.0),
        problem=dict(sigma_eph=0.06, sigma_pp=0.006, nsigma=5.0, hw_cut=0.0002),
        init=dict(T_el=2000.0, T_ph=300.0, mu=0.3),
        seed_offset=12,
    ),
    # Silicon-like 3D bulk: 40^3 simple-cubic-indexed k = q grid, 4 conduction
    # bands (offset cosine bands) in a window 0.4 eV above the band minimum,
    # 6 branches (acoustic TA1/TA2/LA with sin dispersions to 25/27/60 meV,
    # optical near 62-64 meV), sigma 5 meV (e-ph) / 1.1 meV (ph-ph), cutoff
    # 0.2 meV (Methods, silicon grids).  q-point triplets are thinned to ~3%
    # (~2e9 ph-ph channels).  |g|^2 is scaled for an e-ph spectral radius of
    # ~0.5/fs (fast steps of ~1 fs), |V3|^2 for a mean 300 K phonon decay rate
    # of ~1/ps.  Carriers at 2000 K with 0.0184 electrons per cell, phonons at
    # 300 K.
    "si3d": dict(
        grid=dict(dim=3, L=40, lattice=2, n_bands=4, n_modes=6, t_hop=0.5,
                  win_lo=-1.0, win_hi=0.4, with_eph=1, with_pp=1,
                  shell_eph=0.030, shell_pp=0.0066, keep_eph=1.0, keep_pp=1.0, keep_pp_q=0.03,
                  g2_mu=-6.2, g2_sig=1.0, v2_mu=-15.0, v2_sig=1.0),
        problem=dict(sigma_eph=0.005, sigma_pp=0.0011, nsigma=6.0, hw_cut=0.0002),
        init=dict(T_el=2000.0, T_ph=300.0, density=0.0184),
        seed_offset=3,
    ),
    # Integer-lattice toy: every energy is a multiple of 25 meV and only exactly
    # energy-conserving channels are stored (the shell and the n*sigma
    # truncation are both below one quantum).
    "lattice2d": dict(
        grid=dict(dim=2, L=6, lattice=1, n_bands=2, n_modes=6, t_hop=0.08,
                  win_lo=-10.0, win_hi=10.0, with_eph=1, with_pp=1, quantize=1, quantum=0.025,
                  shell_eph=0.005, shell_pp=0.005, keep_eph=1.0, keep_pp=1.0,
                  g2_mu=-4.0, g2_sig=1.0, v2_mu=-10.0, v2_sig=1.0),
        problem=dict(sigma_eph=0.002, sigma_pp=0.002, nsigma=2.0, hw_cut=0.001),
        init=dict(T_el=1500.0, T_ph=1500.0, mu=0.0),
        seed_offset=13,
    ),
}


@dataclass
class Workload:
    name: str
    params: dict
    n_el: int
    n_ph: int
    n_k_total: int
    n_q_total: int
    eps: np.ndarray
    hw: np.ndarray
    el_k: np.ndarray
    el_band: np.ndarray
    el_of_full: np.ndarray
    eph_row: np.ndarray
    eph_partner: np.ndarray
    eph_phonon: np.ndarray
    eph_g2: np.ndarray
    pp_row: np.ndarray
    pp_a: np.ndarray
    pp_b: np.ndarray
    pp_v2: np.ndarray
    sigma_eph: float
    sigma_pp: float
    nsigma: float
    hw_cut: float
    y0: np.ndarray
    grid: dict = field(default_factory=dict)
    init: dict = field(default_factory=dict)

    @property
    def n_y(self) -> int:
        return self.n_el + self.n_ph

    def pp_model(self) -> dict:
        """How the generator drew |V3|^2 (the rtbte_pp_model fields): phonon
        id = q * n_modes + nu over the L^dim grid, Philox4x32-10 keyed by the
        seed's low and high words over the canonical sorted triplet ids and
        the ph-ph stream word, Box-Muller normal, lognormal(v2_mu, v2_sig)."""
        g, seed = self.grid, int(self.params["seed"])
        return dict(dim=int(g["dim"]), L=int(g["L"]), n_modes=int(g["n_modes"]),
                    key0=seed & 0xFFFFFFFF, key1=(seed >> 32) & 0xFFFFFFFF, stream=STREAM_PP,
                    ln_mu=float(g["v2_mu"]), ln_sigma=float(g["v2_sig"]))

    def problem_arrays(self) -> dict:
        """The arrays and scalars the collision-integral problem is stated in."""
        return dict(n_el=self.n_el, n_ph=self.n_ph, n_k_total=self.n_k_total,
                    n_q_total=self.n_q_total, eps=self.eps, hw=self.hw,
                    eph_row=self.eph_row, eph_partner=self.eph_partner,
                    eph_phonon=self.eph_phonon, eph_g2=self.eph_g2,
                    pp_row=self.pp_row, pp_a=self.pp_a, pp_b=self.pp_b, pp_v2=self.pp_v2,
                    sigma_eph=self.sigma_eph, sigma_pp=self.sigma_pp,
                    nsigma=self.nsigma, hw_cut=self.hw_cut)


def make_params(grid: dict, seed: int) -> Params:
    p = Params()
    defaults = dict(quantize=0, quantum=0.025, keep_pp_q=1.0)
    for k, v in {**defaults, **grid}.items():
        setattr(p, k, v)
    p.seed = seed
    return p


def generate(grid: dict, problem: dict, init: dict, seed: int, name: str = "custom",
             dense: bool = False):
    """Enumerate one workload.  Returns a Workload (and dense tables if asked)."""
    L = _lib()
    p = make_params(grid, seed)
    h = L.synth_create(ctypes.byref(p))
    try:
        sizes = np.zeros(6, dtype=np.int64)
        L.synth_sizes(h, _ptr(sizes))
        n_el, n_ph, N, n_eph, n_pp, n_full = (int(x) for x in sizes)
        eps = np.zeros(n_el); el_k = np.zeros(n_el, np.int32); el_band = np.zeros(n_el, np.int32)
        hw = np.zeros(n_ph); el_of_full = np.zeros(n_full, np.int32)
        L.synth_states(h, _ptr(eps), _ptr(el_k), _ptr(el_band), _ptr(hw), _ptr(el_of_full))
        eph = [np.zeros(n_eph, np.int32) for _ in range(3)] + [np.zeros(n_eph)]
        if n_eph:
            L.synth_fill_eph(h, *(_ptr(a) for a in eph))
        pp = [np.zeros(n_pp, np.int32) for _ in range(3)] + [np.zeros(n_pp)]
        if n_pp:
            L.synth_fill_pp(h, *(_ptr(a) for a in pp))
        tables = None
        if dense:
            nb, nm = grid["n_bands"], grid["n_modes"]
            g2d = np.zeros(n_full * nb * nm * N)
            v2d = np.zeros(n_ph * N * nm * nm)
            L.synth_dense(h, _ptr(g2d), _ptr(v2d))
            tables = dict(g2=g2d.reshape(n_full, nb, nm, N),
                          v2=v2d.reshape(n_ph, N, nm, nm))
    finally:
        L.synth_destroy(h)
    mu = init.get("mu", 0.0)
    if "density" in init:   # carriers per cell: sum_window f / N_k = density
        mu = solve_mu(eps, init.get("T_el", 300.0), init["density"], N)
    f0 = fermi_dirac(eps, init.get("T_el", 300.0), mu)
    n0 = bose_einstein(hw, init.get("T_ph", 300.0))
    wl = Workload(name=name, params=dict(grid=grid, problem=problem, init=init, seed=seed),
                  n_el=n_el, n_ph=n_ph, n_k_total=N, n_q_total=N, eps=eps, hw=hw,
                  el_k=el_k, el_band=el_band, el_of_full=el_of_full,
                  eph_row=eph[0], eph_partner=eph[1], eph_phonon=eph[2], eph_g2=eph[3],
                  pp_row=pp[0], pp_a=pp[1], pp_b=pp[2], pp_v2=pp[3],
                  sigma_eph=problem["sigma_eph"], sigma_pp=problem["sigma_pp"],
                  nsigma=problem["nsigma"], hw_cut=problem["hw_cut"],
                  y0=np.concatenate([f0, n0]), grid=dict(grid), init=dict(init))
    return (wl, tables) if dense else wl


def build(name: str, seed: int | None = None, dense: bool = False, **overrides):
    """Build a named workload.  `overrides` replace grid/problem/init keys."""
    r = RECIPES[name]
    grid, problem, init = dict(r["grid"]), dict(r["problem"]), dict(r["init"])
    for k, v in overrides.items():
        for d in (grid, problem, init):
            if k in d:
                d[k] = v
                break
        else:
            grid[k] = v
    if seed is None:
        seed = MASTER_SEED + r.get("seed_offset", 0)
    return generate(grid, problem, init, seed, name=name, dense=dense)


def build_batch(n: int = 64, L_range=(24, 72), T_range=(500.0, 3000.0), recipe: str = "graphene2d",
                seed: int | None = None, **overrides):
    """Independent instances of a recipe for batched runs: instance i has grid
    side L_i drawn uniformly from the integers in L_range and initial electron
    temperature T_i uniformly from T_range (phonons as in the recipe), and its
    own generator seed.  Returns the list of Workloads."""
    if seed is None:
        seed = MASTER_SEED + 5
    rng = np.random.default_rng(seed)
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=n)
    Ts = rng.uniform(T_range[0], T_range[1], size=n)
    return [build(recipe, seed=seed * 1000 + i, L=int(L), T_el=float(T), **overrides)
            for i, (L, T) in enumerate(zip(Ls, Ts))]
