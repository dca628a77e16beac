"""ctypes binding of librtbte.so with the names of the C ABI (include/rtbte.h).

Device buffers are torch CUDA tensors (float64, contiguous) or raw integer
device pointers; streams are torch streams or raw handles.  PyTorch supplies
device memory and streams only: every step of the computation runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

OK, E_INVAL, E_NOMEM, E_HIP, E_STEP, E_NONFINITE, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PART_EPH, PART_PHE, PART_PHPH, PART_ALL = 1, 2, 4, 7
FP64, MIXED = 0, 1
# weight formats of MIXED (rtbte.h): automatic, packed 8-byte words, FP16 + 11-bit tail,
# FP16, BF16 for e-ph / FP16 for ph-ph
W_AUTO, W_PACK8, W_F16X, W_F16, W_BF16_EPH = 0, 1, 2, 3, 4
HEALTH_F_RANGE, HEALTH_N_NEGATIVE = 1, 2
# FP64 channel layouts (rtbte.h)
F64_AUTO, F64_PACKED, F64_PLAIN = 0, 1, 2

_STATUS = {E_INVAL: "invalid argument", E_NOMEM: "out of memory", E_HIP: "HIP error",
           E_STEP: "step failure", E_NONFINITE: "non-finite state", E_UNSUPPORTED: "unsupported"}


class RtbteError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rtbte status {code} ({_STATUS.get(code, '?')}): {msg}")
        self.code = code


class Problem(ctypes.Structure):
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


class PpModel(ctypes.Structure):
    """rtbte_pp_model: the ph-ph matrix elements as a function of the triplet."""
    _fields_ = [("dim", ctypes.c_int32), ("L", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("key0", ctypes.c_uint32), ("key1", ctypes.c_uint32), ("stream", ctypes.c_uint32),
                ("ln_mu", ctypes.c_double), ("ln_sigma", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("mixed_weights", ctypes.c_int32), ("device", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("atol_el", ctypes.c_double), ("atol_ph", ctypes.c_double),
        ("fast_mode", ctypes.c_int32), ("h_fast", ctypes.c_double),
        ("fast_rtol", ctypes.c_double), ("fast_atol_el", ctypes.c_double),
        ("fast_atol_ph", ctypes.c_double),
        ("pid_k1", ctypes.c_double), ("pid_k2", ctypes.c_double), ("pid_k3", ctypes.c_double),
        ("pid_order", ctypes.c_int32), ("pid_alt_sign", ctypes.c_int32),
        ("safety", ctypes.c_double), ("eta_max", ctypes.c_double),
        ("eta_max_first", ctypes.c_double), ("eta_fail_min", ctypes.c_double),
        ("eta_fail_max", ctypes.c_double), ("eps_floor", ctypes.c_double),
        ("max_fails", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("steps_per_poll", ctypes.c_int32), ("group_rows_el", ctypes.c_int32),
        ("group_rows_ph", ctypes.c_int32), ("item_channels", ctypes.c_int64),
        ("tune", ctypes.c_int32), ("tune_cache", ctypes.c_char_p),
        ("fp64_layout", ctypes.c_int32),
        ("fp64_check", ctypes.c_int32),
        ("small_nef", ctypes.c_int32),
        ("eta_fail_repeat", ctypes.c_double),
        ("pp_fold", ctypes.c_int32), ("tiled", ctypes.c_int32), ("pp_model", ctypes.c_void_p),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_rhs_eph", ctypes.c_int64), ("n_rhs_phe", ctypes.c_int64), ("n_rhs_phph", ctypes.c_int64),
        ("n_accept", ctypes.c_int64), ("n_reject", ctypes.c_int64),
        ("n_fast_accept", ctypes.c_int64), ("n_fast_reject", ctypes.c_int64),
        ("t", ctypes.c_double), ("h_last", ctypes.c_double), ("h_min", ctypes.c_double),
        ("h_max", ctypes.c_double), ("eps_last", ctypes.c_double), ("status", ctypes.c_int32),
        ("err_vs_fp64_last", ctypes.c_double), ("health", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None
_vp = ctypes.c_void_p


def lib_path() -> str:
    return os.path.join(HERE, "librtbte.so")


def load():
    """Load librtbte.so; raises if it is not built (there is no fallback)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() "
                           "(the HIP library is required; there is no CPU fallback)")
    L = ctypes.CDLL(path)
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.rtbte_default_options.argtypes = [ctypes.POINTER(Options)]
    L.rtbte_create.argtypes = [ctypes.POINTER(Problem), i32, ctypes.POINTER(Options), ctypes.POINTER(_vp)]
    L.rtbte_destroy.argtypes = [_vp]
    L.rtbte_last_error.argtypes = [_vp]
    L.rtbte_last_error.restype = ctypes.c_char_p
    L.rtbte_layout.argtypes = [_vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.rtbte_ny.argtypes = [_vp]
    L.rtbte_ny.restype = i64
    L.rtbte_counts.argtypes = [_vp, i32, ctypes.POINTER(i64)]
    L.rtbte_stored_counts.argtypes = [_vp, i32, ctypes.POINTER(i64)]
    L.rtbte_rhs.argtypes = [_vp, _vp, _vp, i32, _vp]
    L.rtbte_rhs_noalloc.argtypes = [_vp, _vp, _vp, i32, _vp]
    L.rtbte_noalloc_scratch_bytes.argtypes = [_vp]
    L.rtbte_noalloc_scratch_bytes.restype = i64
    L.rtbte_noalloc_scratch_limit.argtypes = []
    L.rtbte_noalloc_scratch_limit.restype = i64
    L.rtbte_rates.argtypes = [_vp, _vp, _vp, i32, _vp]
    L.rtbte_check_fp64.argtypes = [_vp, _vp, _vp, _vp]
    L.rtbte_energy_average.argtypes = [_vp, _vp, _vp, i32, i32, dbl, dbl, i32, _vp, _vp]
    L.rtbte_mode_temperatures.argtypes = [_vp, _vp, i32, _vp, i32, _vp, _vp]
    L.rtbte_step_adaptive.argtypes = [_vp, _vp, _vp, _vp, dbl, i32, _vp]
    L.rtbte_step_rk4.argtypes = [_vp, _vp, _vp, dbl, i64, _vp]
    L.rtbte_step_multirate.argtypes = [_vp, _vp, _vp, _vp, dbl, dbl, i32, _vp]
    L.rtbte_step_multirate_adaptive.argtypes = [_vp, _vp, _vp, _vp, _vp, dbl, i32, _vp]
    L.rtbte_step_split.argtypes = [_vp, _vp, _vp, dbl, dbl, dbl, _vp]
    L.rtbte_reset.argtypes = [_vp]
    L.rtbte_get_stats.argtypes = [_vp, i32, ctypes.POINTER(Stats)]
    L.rtbte_get_tuning.argtypes = [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
    L.rtbte_get_tuning_source.argtypes = [_vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.rtbte_graph_launches.argtypes = [_vp]
    L.rtbte_graph_launches.restype = i64
    L.rtbte_get_weight_format.argtypes = [_vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.rtbte_get_state.argtypes = [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]
    L.rtbte_set_state.argtypes = [_vp, _vp, ctypes.c_size_t]
    L.rtbte_profile.argtypes = [_vp, i32]
    L.rtbte_profile_read.argtypes = [_vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    _LIB = L
    return L


def noalloc_scratch_limit() -> int:
    """Size of the static device buffer of rhs_noalloc (bytes)."""
    return int(load().rtbte_noalloc_scratch_limit())


def default_options(**kw) -> Options:
    o = Options()
    load().rtbte_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v.encode() if isinstance(v, str) else v)
    return o


def _dptr(x, n=None, what="buffer"):
    """Device pointer of a torch CUDA float64 tensor (or a raw int pointer)."""
    if isinstance(x, int):
        return x
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float64 and x.is_contiguous()):
        raise TypeError(f"{what} must be a contiguous float64 CUDA tensor")
    if n is not None and x.numel() < n:
        raise ValueError(f"{what} has {x.numel()} elements, needs {n}")
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Context:
    """One rtbte context over one or more instances (problem dicts as produced by
    ``synth.Workload.problem_arrays()``)."""

    def __init__(self, problems, options: Options | None = None, **opt_kw):
        L = load()
        if isinstance(problems, dict):
            problems = [problems]
        n = len(problems)
        arr = (Problem * n)()
        keep = []
        for i, P in enumerate(problems):
            p = arr[i]
            for k in ("n_el", "n_ph", "n_k_total", "n_q_total"):
                setattr(p, k, int(P[k]))
            for k in ("eps", "hw", "eph_g2", "pp_v2"):
                if k == "pp_v2" and P.get(k) is None:   # matrix-free ph-ph weights
                    p.pp_v2 = None
                    continue
                a = np.ascontiguousarray(P[k], dtype=np.float64)
                keep.append(a)
                setattr(p, k, a.ctypes.data)
            for k in ("eph_row", "eph_partner", "eph_phonon", "pp_row", "pp_a", "pp_b"):
                a = np.ascontiguousarray(P[k], dtype=np.int32)
                keep.append(a)
                setattr(p, k, a.ctypes.data)
            p.n_eph = len(P["eph_row"])
            p.n_pp = len(P["pp_row"])
            for k in ("sigma_eph", "sigma_pp", "nsigma", "hw_cut"):
                setattr(p, k, float(P[k]))
        models = opt_kw.pop("pp_model", None)
        self.options = options if options is not None else default_options(**opt_kw)
        if models is not None:
            # one model per instance (a dict of rtbte_pp_model fields, or a list of them)
            if isinstance(models, dict):
                models = [models] * n
            if len(models) != n:
                raise ValueError("pp_model: one model per instance")
            marr = (PpModel * n)()
            for i, m in enumerate(models):
                for k, v in m.items():
                    setattr(marr[i], k, v)
            keep.append(marr)
            self.options.pp_model = ctypes.cast(marr, ctypes.c_void_p).value
        h = _vp()
        rc = L.rtbte_create(arr, n, ctypes.byref(self.options), ctypes.byref(h))
        if rc != OK:
            raise RtbteError(rc, L.rtbte_last_error(None).decode())
        self._h = h
        self.n_inst = n
        self.ny = int(L.rtbte_ny(h))

    # -- helpers
    def _check(self, rc):
        if rc != OK:
            raise RtbteError(rc, load().rtbte_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            load().rtbte_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI
    def layout(self, inst=0):
        off, ne, nph = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(load().rtbte_layout(self._h, inst, ctypes.byref(off), ctypes.byref(ne), ctypes.byref(nph)))
        return off.value, ne.value, nph.value

    def counts(self, inst=-1):
        """Channels the right-hand side sums (e-ph, ph-e, ph-ph), as the method defines them."""
        c = (ctypes.c_int64 * 3)()
        self._check(load().rtbte_counts(self._h, inst, c))
        return tuple(c)

    def stored_counts(self, inst=-1):
        """Channels stored and streamed (fewer ph-ph ones under pp_fold)."""
        c = (ctypes.c_int64 * 3)()
        self._check(load().rtbte_stored_counts(self._h, inst, c))
        return tuple(c)

    def rhs(self, y, ydot, parts=PART_ALL, stream=None):
        self._check(load().rtbte_rhs(self._h, _dptr(y, self.ny, "y"), _dptr(ydot, self.ny, "ydot"),
                                     int(parts), _stream(stream)))

    def rhs_noalloc(self, y, ydot, parts=PART_ALL, stream=None):
        """rhs() with its scratch in the library's static device buffer (no
        allocation; calls that overlap in time on one device race)."""
        self._check(load().rtbte_rhs_noalloc(self._h, _dptr(y, self.ny, "y"), _dptr(ydot, self.ny, "ydot"),
                                             int(parts), _stream(stream)))

    def noalloc_scratch_bytes(self) -> int:
        """Static scratch bytes rhs_noalloc needs for this context."""
        return int(load().rtbte_noalloc_scratch_bytes(self._h))

    def rates(self, y, out, parts=PART_ALL, stream=None):
        """Linearized rates -d(ydot_i)/d(y_i), partners held fixed (FP64 contexts)."""
        self._check(load().rtbte_rates(self._h, _dptr(y, self.ny, "y"), _dptr(out, self.ny, "rates"),
                                       int(parts), _stream(stream)))

    def check_fp64(self, y, stream=None):
        """Per instance ||f_mixed(y) - f_fp64(y)|| / ||f_fp64(y)|| (mixed
        contexts created with fp64_check > 0)."""
        out = np.empty(self.n_inst, dtype=np.float64)
        self._check(load().rtbte_check_fp64(self._h, _dptr(y, self.ny, "y"), out.ctypes.data_as(_vp),
                                            _stream(stream)))
        return out

    def energy_average(self, y, e_lo, e_hi, n_bins, phonons=False, y_ref=None, inst=0, stream=None):
        """Per energy bin: (state count, mean population, mean of y - y_ref)
        of one instance's carriers (phonons=False, binned by eps) or phonons
        (binned by hbar omega); numpy arrays of n_bins each."""
        out = np.empty(3 * int(n_bins), dtype=np.float64)
        ref = None if y_ref is None else _dptr(y_ref, self.ny, "y_ref")
        self._check(load().rtbte_energy_average(self._h, _dptr(y, self.ny, "y"), ref, int(inst), int(bool(phonons)),
                                                float(e_lo), float(e_hi), int(n_bins),
                                                out.ctypes.data_as(_vp), _stream(stream)))
        o = out.reshape(-1, 3)
        return o[:, 0].copy(), o[:, 1].copy(), o[:, 2].copy()

    def mode_temperatures(self, y, mode_of, n_modes, inst=0, stream=None):
        """Effective temperature (K) of each phonon branch of one instance;
        mode_of gives the branch of each of the instance's phonon states."""
        m = np.ascontiguousarray(mode_of, dtype=np.int32)
        if m.shape != (self.layout(inst)[2],):
            raise ValueError(f"mode_of must have one entry per phonon state of instance {inst}")
        out = np.empty(int(n_modes), dtype=np.float64)
        self._check(load().rtbte_mode_temperatures(self._h, _dptr(y, self.ny, "y"), int(inst),
                                                   m.ctypes.data_as(_vp), int(n_modes),
                                                   out.ctypes.data_as(_vp), _stream(stream)))
        return out

    def step_adaptive(self, y, t, h, t_out, one_step=False, stream=None):
        self._check(load().rtbte_step_adaptive(self._h, _dptr(y, self.ny, "y"), _dptr(t, self.n_inst, "t"),
                                               _dptr(h, self.n_inst, "h"), float(t_out), int(bool(one_step)),
                                               _stream(stream)))

    def step_rk4(self, y, t, h_step, n_steps, stream=None):
        self._check(load().rtbte_step_rk4(self._h, _dptr(y, self.ny, "y"), _dptr(t, self.n_inst, "t"),
                                          float(h_step), int(n_steps), _stream(stream)))

    def step_multirate(self, y, t, h_fast, t_out, h_slow, one_step=False, stream=None):
        self._check(load().rtbte_step_multirate(self._h, _dptr(y, self.ny, "y"), _dptr(t, self.n_inst, "t"),
                                                _dptr(h_fast, self.n_inst, "h_fast"), float(t_out), float(h_slow),
                                                int(bool(one_step)), _stream(stream)))

    def step_multirate_adaptive(self, y, t, h_fast, h_slow, t_out, one_step=False, stream=None):
        """MIS with the slow step chosen by step doubling; h_slow (device, one
        entry per instance, all equal: the slow steps are common) holds the
        first slow step and receives the next one."""
        n = self.n_inst
        self._check(load().rtbte_step_multirate_adaptive(self._h, _dptr(y, self.ny, "y"), _dptr(t, n, "t"),
                                                         _dptr(h_fast, n, "h_fast"), _dptr(h_slow, n, "h_slow"),
                                                         float(t_out), int(bool(one_step)), _stream(stream)))

    def step_split(self, y, t, h_fast, h_slow, t_out, stream=None):
        self._check(load().rtbte_step_split(self._h, _dptr(y, self.ny, "y"), _dptr(t, self.n_inst, "t"), float(h_fast),
                                            float(h_slow), float(t_out), _stream(stream)))

    def reset(self):
        self._check(load().rtbte_reset(self._h))

    def stats(self, inst=0) -> dict:
        s = Stats()
        self._check(load().rtbte_get_stats(self._h, inst, ctypes.byref(s)))
        return s.as_dict()

    def tuning(self):
        """(electron rows per group, phonon rows per group, channels per item)."""
        ge, gp, ic = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        self._check(load().rtbte_get_tuning(self._h, ctypes.byref(ge), ctypes.byref(gp), ctypes.byref(ic)))
        return ge.value, gp.value, ic.value

    def tuning_source(self):
        """(0 given/default, 1 tuned at create, 2 from the tune cache; measured ms per RHS)."""
        src, ms = ctypes.c_int32(), ctypes.c_double()
        self._check(load().rtbte_get_tuning_source(self._h, ctypes.byref(src), ctypes.byref(ms)))
        return src.value, ms.value

    def weight_format(self):
        """(RTBTE_W_* format or -1 for FP64, bytes per channel, relative rounding of a stored weight)."""
        f, b, u = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self._check(load().rtbte_get_weight_format(self._h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(u)))
        return f.value, b.value, u.value

    def graph_launches(self) -> int:
        return int(load().rtbte_graph_launches(self._h))

    def profile(self, enable=True):
        self._check(load().rtbte_profile(self._h, int(bool(enable))))

    def profile_read(self):
        """(summed collision-kernel ms, launches, summed algorithmic bytes)."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._check(load().rtbte_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(by)))
        return ms.value, n.value, by.value

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        self._check(load().rtbte_get_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(load().rtbte_get_state(self._h, buf, ctypes.byref(n)))
        return buf.raw[:n.value]

    def set_state(self, data: bytes):
        buf = ctypes.create_string_buffer(data, len(data))
        self._check(load().rtbte_set_state(self._h, buf, len(data)))
