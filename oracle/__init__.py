"""FP64 CPU oracle for the rt-BTE hot path.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only permitted users.  The product
path (the HIP library and its binding) never imports, links or runs anything
here, and nothing here imports the product.

* ``rtbte_oracle.c`` (built to ``liboracle.so``) evaluates the collision
  integrals of Methods Eq. (e-ph) and Eq. (ph-ph) over the stored channel
  lists with compensated row sums, and by brute force over dense tables on
  tiny grids.
* ``integrators.py`` advances Eq. (erk_ode) with the classical RK4, the
  adaptive Zonneveld 4(3) ERK with WRMS norm and PID control (Methods,
  ERK method), and the third-order MIS multirate method (Methods, MRI method).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

PART_EPH, PART_PHE, PART_PHPH, PART_ALL = 1, 2, 4, 7


# RTBTE_HOST_SANITIZE=1 selects a build of the same source under
# AddressSanitizer and UndefinedBehaviorSanitizer (host code only; the
# process must preload the sanitizer runtimes).
_SANITIZE = os.environ.get("RTBTE_HOST_SANITIZE") == "1"
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                  "-fno-omit-frame-pointer", "-g"]


def lib_path(sanitized=None) -> str:
    san = _SANITIZE if sanitized is None else sanitized
    return os.path.join(_HERE, "liboracle_san.so" if san else "liboracle.so")


def build_lib(sanitized=None) -> str:
    """Compile rtbte_oracle.c (plain C, OpenMP, no fast-math, no FMA
    contraction); with sanitized (default: RTBTE_HOST_SANITIZE) into
    liboracle_san.so under ASan and UBSan."""
    import subprocess
    san = _SANITIZE if sanitized is None else sanitized
    out = lib_path(san)
    cmd = (["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall"] + (SANITIZE_FLAGS if san else []) +
           ["-o", out + ".tmp", os.path.join(_HERE, "rtbte_oracle.c"), "-lm"])
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_el", ctypes.c_int32), ("n_ph", ctypes.c_int32),
        ("n_k_total", ctypes.c_int32), ("n_q_total", ctypes.c_int32),
        ("eps", ctypes.c_void_p), ("hw", ctypes.c_void_p),
        ("n_eph", ctypes.c_int64),
        ("eph_row", ctypes.c_void_p), ("eph_partner", ctypes.c_void_p),
        ("eph_phonon", ctypes.c_void_p), ("eph_g2", ctypes.c_void_p),
        ("n_pp", ctypes.c_int64),
        ("pp_row", ctypes.c_void_p), ("pp_a", ctypes.c_void_p), ("pp_b", ctypes.c_void_p),
        ("pp_v2", ctypes.c_void_p),
        ("sigma_eph", ctypes.c_double), ("sigma_pp", ctypes.c_double),
        ("nsigma", ctypes.c_double), ("hw_cut", ctypes.c_double),
    ]


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path()):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(lib_path())
        L.orc_build.restype = ctypes.c_void_p
        L.orc_build.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_int)]
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_counts.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_rates.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        L.orc_max_weight.argtypes = [ctypes.c_void_p]
        L.orc_max_weight.restype = ctypes.c_double
        L.orc_rhs_rows.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_brute_rhs.argtypes = ([ctypes.c_int] * 7 + [ctypes.c_void_p] * 5 +
                                    [ctypes.c_double] * 4 + [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int])
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def threads() -> int:
    return int(_lib().orc_threads())


def set_threads(n: int) -> None:
    """Thread count of the oracle's OpenMP loops."""
    _lib().orc_set_threads(int(n))


class Oracle:
    """Weighted channel lists of one problem, and its right-hand side."""

    def __init__(self, prob: dict):
        self._keep = {}
        P = _Problem()
        for k in ("n_el", "n_ph", "n_k_total", "n_q_total"):
            setattr(P, k, int(prob[k]))
        for k in ("eps", "hw", "eph_g2", "pp_v2"):
            a = np.ascontiguousarray(prob[k], dtype=np.float64)
            self._keep[k] = a
            setattr(P, k, a.ctypes.data)
        for k in ("eph_row", "eph_partner", "eph_phonon", "pp_row", "pp_a", "pp_b"):
            a = np.ascontiguousarray(prob[k], dtype=np.int32)
            self._keep[k] = a
            setattr(P, k, a.ctypes.data)
        P.n_eph = len(self._keep["eph_row"])
        P.n_pp = len(self._keep["pp_row"])
        for k in ("sigma_eph", "sigma_pp", "nsigma", "hw_cut"):
            setattr(P, k, float(prob[k]))
        st = ctypes.c_int(0)
        self._h = _lib().orc_build(ctypes.byref(P), ctypes.byref(st))
        if not self._h:
            raise ValueError(f"oracle build failed (status {st.value})")
        self._keep = None  # the lists hold their own copies
        self.n_el = int(prob["n_el"])
        self.n_ph = int(prob["n_ph"])
        self.n_y = self.n_el + self.n_ph

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib().orc_free(h)
            self._h = None

    def counts(self):
        """Stored channels (C_e electron-side e-ph, C_pe phonon-side ph-e, C_pp ph-ph)."""
        out = np.zeros(3, dtype=np.int64)
        _lib().orc_counts(self._h, _p(out))
        return tuple(int(x) for x in out)

    def rhs(self, y, parts: int = PART_ALL, scales: bool = False, unweighted: bool = False):
        """f(y) restricted to `parts`.  With scales=True also returns, per row,
        S = sum |W F| and A = sum |W| (|gain| + |loss|); with unweighted=True
        additionally M = sum (|gain| + |loss|) and Q = sum (W F)^2."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert y.shape == (self.n_y,)
        out = np.empty(self.n_y)
        S = np.empty(self.n_y) if scales else None
        A = np.empty(self.n_y) if scales else None
        M = np.empty(self.n_y) if unweighted else None
        Q = np.empty(self.n_y) if unweighted else None
        _lib().orc_rhs(self._h, _p(y), _p(out), int(parts), _p(S), _p(A), _p(M), _p(Q))
        if unweighted:
            return out, S, A, M, Q
        return (out, S, A) if scales else out

    def rates(self, y, parts: int = PART_ALL, magnitude: bool = False):
        """Linearized rates -d(ydot_i)/d(y_i) of the parts in `parts`, partner
        populations held fixed; with magnitude=True also sum |W|(|X|+|Y|)."""
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert y.shape == (self.n_y,)
        out = np.empty(self.n_y)
        mag = np.empty(self.n_y) if magnitude else None
        _lib().orc_rates(self._h, _p(y), _p(out), int(parts), _p(mag))
        return (out, mag) if magnitude else out

    def max_weight(self) -> float:
        """Largest stored channel weight."""
        return float(_lib().orc_max_weight(self._h))

    def rhs_rows(self, y, rows, parts: int = PART_ALL):
        y = np.ascontiguousarray(y, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        assert rows.min(initial=0) >= 0 and rows.max(initial=0) < self.n_y
        out = np.empty(len(rows)); S = np.empty(len(rows)); A = np.empty(len(rows))
        _lib().orc_rhs_rows(self._h, _p(y), _p(rows), len(rows), _p(out), int(parts), _p(S), _p(A))
        return out, S, A


def brute_rhs(wl, tables: dict, y, parts: int = PART_ALL):
    """Direct grid sums of Eq. (e-ph) and Eq. (ph-ph) from dense tables (tiny grids)."""
    g = wl.grid
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty(wl.n_y)
    g2 = np.ascontiguousarray(tables["g2"], dtype=np.float64)
    v2 = np.ascontiguousarray(tables["v2"], dtype=np.float64)
    eof = np.ascontiguousarray(wl.el_of_full, dtype=np.int32)
    _lib().orc_brute_rhs(int(g["dim"]), int(g["L"]), int(g["n_bands"]), int(g["n_modes"]),
                         int(wl.n_k_total), int(wl.n_q_total), int(wl.n_el), _p(eof),
                         _p(np.ascontiguousarray(wl.eps)), _p(np.ascontiguousarray(wl.hw)),
                         _p(g2), _p(v2), float(wl.sigma_eph), float(wl.sigma_pp),
                         float(wl.nsigma), float(wl.hw_cut), _p(y), _p(out), int(parts))
    return out
