"""The C ABI used from plain C: the example program (built with the
library) reads a problem and a state, evaluates the right-hand side on the
GPU into caller-owned device buffers and writes it back; the result matches
the oracle on every row (1e-12 A_i) and the channel counts are the oracle's.
Given an end time it also runs the adaptive ERK, bitwise as the binding does."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import say, to_dev, torch_cuda
from tests.test_gpu_rhs import random_state

pytestmark = pytest.mark.gpu


def write_problem(d, prob, y):
    with open(os.path.join(d, "meta.txt"), "w") as f:
        f.write(" ".join(str(x) for x in (prob["n_el"], prob["n_ph"], prob["n_k_total"], prob["n_q_total"],
                                         len(prob["eph_row"]), len(prob["pp_row"]))) + " ")
        f.write(" ".join(repr(float(prob[k])) for k in ("sigma_eph", "sigma_pp", "nsigma", "hw_cut")) + "\n")
    for k in ("eps", "hw", "eph_g2", "pp_v2"):
        np.ascontiguousarray(prob[k], dtype="<f8").tofile(os.path.join(d, k + ".f64"))
    for k in ("eph_row", "eph_partner", "eph_phonon", "pp_row", "pp_a", "pp_b"):
        np.ascontiguousarray(prob[k], dtype="<i4").tofile(os.path.join(d, k + ".i32"))
    np.ascontiguousarray(y, dtype="<f8").tofile(os.path.join(d, "y.f64"))


@pytest.mark.parametrize("name", ["tiny2d", "tiny3d"])
def test_c_example_matches_oracle(name, tmp_path):
    torch_cuda()
    from paper_2412_13402_amd import build
    if not os.path.exists(build.EXAMPLE):
        pytest.fail("the C example is not built (run __graft_entry__.build())")
    wl = synth.build(name)
    prob = wl.problem_arrays()
    y = random_state(wl, 31)
    write_problem(str(tmp_path), prob, y)
    say(f"[c] example_rhs {name}")
    r = subprocess.run([build.EXAMPLE, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    g = np.fromfile(os.path.join(str(tmp_path), "ydot.f64"), dtype="<f8")
    o = oracle.Oracle(prob)
    ref, S, A = o.rhs(y, scales=True)
    assert g.shape == ref.shape and np.all(np.abs(g - ref) <= 1e-12 * A + 1e-300)
    assert tuple(int(x) for x in r.stdout.split()) == o.counts()


def test_c_example_steps_as_the_binding_does(tmp_path):
    """The C program's adaptive ERK run (default options, library-chosen
    starting step, 0 -> 5 fs) is bitwise the one the Python binding makes on
    the same inputs, with the same accepted and rejected steps."""
    torch = torch_cuda()
    import paper_2412_13402_amd as P
    from paper_2412_13402_amd import build
    if not os.path.exists(build.EXAMPLE):
        pytest.fail("the C example is not built (run __graft_entry__.build())")
    wl = synth.build("tiny2d")
    prob = wl.problem_arrays()
    write_problem(str(tmp_path), prob, wl.y0)
    say("[c] example_rhs tiny2d, ERK to 5 fs")
    r = subprocess.run([build.EXAMPLE, str(tmp_path), "5.0"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    got = np.fromfile(os.path.join(str(tmp_path), "y_out.f64"), dtype="<f8")
    acc, rej = (int(v) for v in r.stdout.split("\n")[1].split())
    ctx = P.Context(prob)
    y = to_dev(wl.y0)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    h = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.step_adaptive(y, t, h, 5.0)
    torch.cuda.synchronize()
    st = ctx.stats()
    assert np.array_equal(got, y.cpu().numpy())
    assert (acc, rej) == (st["n_accept"], st["n_reject"]) and acc >= 2
