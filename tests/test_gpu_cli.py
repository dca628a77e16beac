"""The command-line drivers end to end on a small workload: every method of
the run driver reaches the end time, conserves the carrier number (e-ph
scattering moves carriers between states only) and reports branch
temperatures."""
import json

import numpy as np
import pytest

from tests.gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu


# on tiny2d both parts relax at up to ~4/fs (largest linearized rates at the
# initial state): fixed steps stay well inside the explicit methods'
# stability limits (about 0.7 fs), checked with the oracle's integrators
@pytest.mark.parametrize("method,extra", [("erk", []), ("rk4", ["--h", "0.1"]),
                                          ("mis", ["--h-slow", "0.5", "--h-fast", "0.1"]),
                                          ("mis-adaptive", ["--h-slow", "0.5", "--h-fast", "0"])])
def test_run_driver(method, extra, capsys):
    torch_cuda()
    from paper_2412_13402_amd import run
    import synth
    say(f"[cli] run {method}")
    res = run.main(["--workload", "tiny2d", "--method", method, "--t-end", "40", "--checks", "2"] + extra)
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["t_end_fs"] == 40.0 and res["history"][-1]["t_fs"] == 40.0
    wl = synth.build("tiny2d")
    n0 = float(wl.y0[:wl.n_el].sum())
    assert abs(res["history"][-1]["carriers"] - n0) <= 1e-9 * n0
    T = res["history"][-1]["phonon_T_K"]
    assert len(T) == wl.grid["n_modes"] and all(np.isfinite(T)) and all(x > 0 for x in T)
    assert out["health"] == 0          # occupations stayed in their physical range


@pytest.mark.parametrize("method,extra", [("erk", []), ("mis-adaptive", ["--h-slow", "0.5", "--h-fast", "0"])])
def test_run_driver_batch(method, extra, capsys):
    """A batch of three small graphene-like instances through the run driver:
    every instance reaches the end time and keeps its carrier number."""
    torch_cuda()
    from paper_2412_13402_amd import run
    import synth
    say(f"[cli] run --batch 3 {method}")
    res = run.main(["--workload", "graphene2d", "--batch", "3", "--batch-L", "8", "12", "--method", method,
                    "--t-end", "20", "--checks", "2"] + extra)
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["n_inst"] == 3 and len(out["steps"]) == 3 and out["health"] == [0, 0, 0]
    ws = synth.build_batch(3, (8, 12), (500.0, 3000.0))
    last = res["history"][-1]["instances"]
    for w, e in zip(ws, last):
        assert e["t_fs"] == 20.0
        n0 = float(w.y0[:w.n_el].sum())
        assert abs(e["carriers"] - n0) <= 1e-9 * n0
        assert all(np.isfinite(e["phonon_T_K"])) and all(x > 0 for x in e["phonon_T_K"])
