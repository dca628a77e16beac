"""The error-versus-cost harness on a small coupled problem (fast e-ph,
slow ph-ph, random populations): every method's error must fall as its
parameter is refined, at the rate its order predicts where the rate is
clean (RK4 ~4, MRI ~3, operator splitting ~1), and the cost counters must
match the method (one ph-ph evaluation per RK4 stage; three per MRI slow
step); the adaptive slow step takes more steps at tighter tolerances."""
import numpy as np
import pytest

from tests.gpu_util import say, torch_cuda
from tests.test_gpu_integrators import coupled

pytestmark = pytest.mark.gpu


def test_error_cost_trends():
    torch_cuda()
    from paper_2412_13402_amd.error_cost import Harness
    Pr, y0 = coupled()
    H = Harness(Pr, y0, Pr["n_el"], 40.0, 4)
    say("[error-cost] reference MRI h_s = 0.05 fs")
    H.reference(hs=0.05)
    rk = [H.rk4(h) for h in (2.0, 1.0, 0.5)]
    er = [H.erk(r, history=(r == 1e-7)) for r in (1e-5, 1e-7, 1e-9)]
    mr = [H.mri(hs, r) for hs, r in ((5.0, 1e-9), (2.5, 1e-10), (1.25, 1e-11))]
    sp = [H.split(0.1, hs) for hs in (2.0, 1.0)]
    ma = [H.mri_adaptive(r) for r in (1e-5, 1e-7, 1e-9)]
    for rows in (rk, er, mr, sp, ma):
        e = [r["err_carriers"] + r["err_phonons"] for r in rows]
        say("    " + rows[0]["method"] + ": " + ", ".join(f"{x:.2e}" for x in e))
        assert all(a > b for a, b in zip(e, e[1:]))
    order = lambda rows: np.log2(rows[0]["err_phonons"] / rows[1]["err_phonons"])
    assert 3.4 < order(rk) < 4.6
    assert 2.4 < order(mr) < 3.6
    assert 0.7 < order(sp) < 1.4
    assert rk[0]["rhs_phph"] == 4 * 20 and mr[0]["rhs_phph"] == 3 * 8
    assert ma[0]["slow_accept"] < ma[1]["slow_accept"] < ma[2]["slow_accept"]
    assert er[1]["step_history"] and abs(er[1]["step_history"][-1][0] - 40.0) < 1e-12
