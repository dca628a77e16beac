"""Error versus cost of the time integrators on one workload (Results, Fig. 2
and Fig. 3 of the paper, on seeded synthetic inputs).

Every method advances the same initial state to t_end on the GPU; the
population errors ||f - f_ref|| / ||f_ref|| (carriers) and
||N - N_ref|| / ||N_ref|| (phonons) are taken against a reference solution
computed, as in the paper (Methods, choices of tolerances and reference
solutions), with the MRI method at a very small slow step and tight fast
tolerances.  Cost is GPU wall time and the number of right-hand-side
evaluations of each part (the ph-ph evaluations drive the cost).

Methods and parameter sweeps (as in the paper's Fig. 2 and Fig. 3):
  RK4    fixed h from 5 fs down to 0.01 fs;
  ERK    adaptive Zonneveld, rtol 1e-4 .. 1e-11, atol 1e-15 for both parts;
  MRI    MIS with an adaptive ERK fast solver, slow step h_s from 20 fs down
         to 0.05 fs paired with fast rtol 1e-4 .. 1e-11 (atol 1e-9 carriers,
         1e-12 phonons);
  split  first-order operator splitting with RK4: e-ph 0.5 fs, ph-ph 5 fs;
  MRI-a  MIS with the slow step chosen by step doubling (the extension the
         paper leaves to future work), rtol 1e-4 .. 1e-9 for the slow step
         and rtol/10 for the adaptive fast solver (atol as for MRI).
Errors are also recorded at intermediate times (Fig. 3) and the step sizes of
the ERK run at rtol 1e-5 (the paper's step-size history).

Run:  python -m paper_2412_13402_amd.error_cost --workload graphene2d --L 48
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

RK4_H = (5.0, 2.0, 1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01)
ERK_RTOL = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10, 1e-11)
MRI_HS = (20.0, 10.0, 5.0, 2.0, 1.0, 0.5, 0.1, 0.05)
MRI_RTOL = ERK_RTOL
SPLIT = ((0.5, 5.0),)
MRIA_RTOL = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9)


def rel_err(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


class Harness:
    """Runs of one problem (problem arrays, initial state y0 = [f; N] with
    n_el carrier components) to t_end, with states kept at n_checks evenly
    spaced times.  Every context replays its step sequence from HIP graphs and
    polls every 2 steps (tiny fast intervals need a step or two each)."""

    def __init__(self, prob, y0, n_el, t_end, n_checks, precision=0, progress=None):
        import torch
        from . import rtbte as R
        self.torch = torch
        self.R = R
        self.prob = prob
        self.y0 = np.asarray(y0, dtype=np.float64)
        self.n_el = int(n_el)
        self.t_end = float(t_end)
        self.checks = [self.t_end * (k + 1) / n_checks for k in range(n_checks)]
        self.precision = precision
        self.ref = None
        self.rows = []
        self.progress = progress    # called with (t, wall) at every check time

    def _ctx(self, **kw):
        return self.R.Context(self.prob, precision=self.precision, use_graph=1, steps_per_poll=2, **kw)

    def _run(self, advance, ctx):
        """Advance through the check times; returns the states there, wall s."""
        torch = self.torch
        dev = torch.device("cuda:0")
        y = torch.tensor(self.y0, dtype=torch.float64, device=dev)
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        h = torch.zeros(1, dtype=torch.float64, device=dev)
        states = []
        torch.cuda.synchronize()
        wall = 0.0
        for tc in self.checks:
            w0 = time.perf_counter()
            advance(ctx, y, t, h, tc)
            torch.cuda.synchronize()
            wall += time.perf_counter() - w0
            states.append(y.cpu().numpy())
            if self.progress:
                self.progress(tc, wall)
        return states, wall

    def reference(self, hs=0.01, rtol=1e-10, atol=1e-15):
        ctx = self._ctx(fast_mode=0, fast_rtol=rtol, fast_atol_el=atol, fast_atol_ph=atol)
        states, wall = self._run(lambda c, y, t, h, tc: c.step_multirate(y, t, h, tc, hs), ctx)
        self.ref = states
        return dict(method="reference (MRI)", h_s=hs, fast_rtol=rtol, atol=atol, wall_s=wall, **self._counts(ctx))

    def _counts(self, ctx):
        st = ctx.stats()
        return dict(rhs_eph=st["n_rhs_eph"], rhs_phph=st["n_rhs_phph"])

    def _record(self, label, params, ctx, states, wall):
        ne = self.n_el
        fin, ref = states[-1], self.ref[-1]
        row = dict(method=label, **params, wall_s=wall, **self._counts(ctx),
                   err_carriers=rel_err(fin[:ne], ref[:ne]), err_phonons=rel_err(fin[ne:], ref[ne:]),
                   err_history=[dict(t_fs=tc, carriers=rel_err(s[:ne], r[:ne]), phonons=rel_err(s[ne:], r[ne:]))
                                for tc, s, r in zip(self.checks, states, self.ref)])
        self.rows.append(row)
        return row

    def rk4(self, h):
        def adv(c, y, t, hh, tc):
            n = int(round((tc - float(t.item())) / h))
            c.step_rk4(y, t, h, n)
        ctx = self._ctx()
        states, wall = self._run(adv, ctx)
        return self._record("RK4", dict(h=h), ctx, states, wall)

    def erk(self, rtol, atol=1e-15, history=False):
        ctx = self._ctx(rtol=rtol, atol_el=atol, atol_ph=atol)
        steps = []
        if history:
            def adv(c, y, t, hh, tc):
                while float(t.item()) < tc:
                    c.step_adaptive(y, t, hh, tc, one_step=True)
                    steps.append((float(t.item()), float(hh.item())))
        else:
            def adv(c, y, t, hh, tc):
                c.step_adaptive(y, t, hh, tc)
        states, wall = self._run(adv, ctx)
        row = self._record("ERK", dict(rtol=rtol, atol=atol), ctx, states, wall)
        if history:
            row["step_history"] = steps
        return row

    def mri(self, hs, rtol, atol_el=1e-9, atol_ph=1e-12):
        ctx = self._ctx(fast_mode=0, fast_rtol=rtol, fast_atol_el=atol_el, fast_atol_ph=atol_ph)
        states, wall = self._run(lambda c, y, t, h, tc: c.step_multirate(y, t, h, tc, hs), ctx)
        return self._record("MRI", dict(h_s=hs, fast_rtol=rtol), ctx, states, wall)

    def mri_adaptive(self, rtol, atol_el=1e-9, atol_ph=1e-12, h_slow0=1.0):
        torch = self.torch
        ctx = self._ctx(fast_mode=0, fast_rtol=0.1 * rtol, fast_atol_el=atol_el, fast_atol_ph=atol_ph,
                        rtol=rtol, atol_el=atol_el, atol_ph=atol_ph)
        hs = torch.full((1,), float(h_slow0), dtype=torch.float64, device="cuda:0")
        states, wall = self._run(lambda c, y, t, h, tc: c.step_multirate_adaptive(y, t, h, hs, tc), ctx)
        st = ctx.stats()
        row = self._record("MRI-adaptive", dict(rtol=rtol, fast_rtol=0.1 * rtol), ctx, states, wall)
        row.update(slow_accept=st["n_accept"], slow_reject=st["n_reject"], h_slow_last=float(hs.item()))
        return row

    def split(self, hf, hs):
        ctx = self._ctx()
        states, wall = self._run(lambda c, y, t, h, tc: c.step_split(y, t, hf, hs, tc), ctx)
        return self._record("split", dict(h_fast=hf, h_slow=hs), ctx, states, wall)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="graphene2d")
    ap.add_argument("--L", type=int, default=48)
    ap.add_argument("--t-end", type=float, default=500.0)
    ap.add_argument("--checks", type=int, default=10, help="error-history points up to t_end")
    ap.add_argument("--ref-hs", type=float, default=0.01)
    ap.add_argument("--rk4-min-h", type=float, default=0.01)
    ap.add_argument("--mri-min-hs", type=float, default=0.05)
    ap.add_argument("--quick", action="store_true", help="a few points per method")
    ap.add_argument("--methods", default="rk4,erk,mri,split,mria",
                    help="comma-separated subset of rk4, erk, mri, split, mria (MRI with adaptive slow step)")
    ap.add_argument("--out", default=None, help="write the JSON result here")
    ap.add_argument("--ref-save", default=None, help="save the reference states (.npz)")
    ap.add_argument("--ref-load", default=None, help="reuse reference states saved by --ref-save")
    a = ap.parse_args(argv)
    import synth
    wl = synth.build(a.workload, L=a.L)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    H = Harness(wl.problem_arrays(), wl.y0, wl.n_el, a.t_end, a.checks,
                progress=lambda tc, w: log(f"    t = {tc:g} fs, {w:.2f} s"))
    log(f"[error-cost] {a.workload} L={a.L}: n_el {wl.n_el} n_ph {wl.n_ph}, to {a.t_end:g} fs")
    res = {"workload": f"{a.workload} L={a.L}", "t_end_fs": a.t_end}
    if a.ref_load:
        z = np.load(a.ref_load)
        H.ref = list(z["states"])
        res["reference"] = json.loads(str(z["meta"]))
        log(f"[error-cost] reference loaded from {a.ref_load}")
    else:
        res["reference"] = H.reference(hs=a.ref_hs)
        log(f"[error-cost] reference in {res['reference']['wall_s']:.1f} s")
        if a.ref_save:
            np.savez(a.ref_save, states=np.array(H.ref), meta=json.dumps(res["reference"]))
    rk4 = [h for h in RK4_H if h >= a.rk4_min_h]
    erk, mri = list(ERK_RTOL), [(h, r) for h, r in zip(MRI_HS, MRI_RTOL) if h >= a.mri_min_hs]
    if a.quick:
        rk4, erk, mri = rk4[::3], erk[::3], mri[::3]
    def attempt(label, fn, *args, **kw):
        try:
            r = fn(*args, **kw)
            log(f"  {label}: {r['wall_s']:.3f} s err {r['err_carriers']:.2e} / {r['err_phonons']:.2e}")
        except H.R.RtbteError as e:   # e.g. an error test that FP64 rounding cannot pass
            H.rows.append(dict(method=label.split()[0], params=label, failed=str(e)))
            log(f"  {label}: failed ({e})")

    methods = set(a.methods.split(","))
    for h in rk4 if "rk4" in methods else ():
        attempt(f"RK4 h={h:g}", H.rk4, h)
    for rt in erk if "erk" in methods else ():
        attempt(f"ERK rtol={rt:g}", H.erk, rt, history=(rt == 1e-5))
    for hs, rt in mri if "mri" in methods else ():
        attempt(f"MRI h_s={hs:g} rtol={rt:g}", H.mri, hs, rt)
    for hf, hs in SPLIT if "split" in methods else ():
        attempt(f"split {hf:g}/{hs:g}", H.split, hf, hs)
    for rt in (MRIA_RTOL[::2] if a.quick else MRIA_RTOL) if "mria" in methods else ():
        attempt(f"MRI-adaptive rtol={rt:g}", H.mri_adaptive, rt)
    res["runs"] = H.rows
    text = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)
    return res


if __name__ == "__main__":
    main()
