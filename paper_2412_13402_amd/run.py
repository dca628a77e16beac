"""Run one workload from its initial state to an end time with one of the
integrators and report wall time, simulated ps per second, the work done and
the effective phonon-branch temperatures at the end.

    python -m paper_2412_13402_amd.run --workload graphene2d --method erk --t-end 10000
    python -m paper_2412_13402_amd.run --workload si3d --method mis --h-slow 50 --h-fast 1 --t-end 20000

Methods: erk (adaptive Zonneveld ERK on the whole right-hand side), rk4
(fixed steps --h), mis (MRI with MIS coupling, slow step --h-slow; fast part
by fixed RK4 steps --h-fast, or by the adaptive ERK with --fast-rtol when
--h-fast is 0), mis-adaptive (the same with the slow step chosen from rtol by
step doubling, starting from --h-slow).  Progress lines go to stderr at
--checks evenly spaced times; one JSON line goes to stdout at the end.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="graphene2d")
    ap.add_argument("--L", type=int, default=None, help="grid side (default: the recipe's)")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--method", choices=("erk", "rk4", "mis", "mis-adaptive"), default="erk")
    ap.add_argument("--t-end", type=float, default=10000.0, help="fs")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--atol-el", type=float, default=1e-9)
    ap.add_argument("--atol-ph", type=float, default=1e-12)
    ap.add_argument("--h", type=float, default=1.0, help="rk4 step (fs)")
    ap.add_argument("--h-slow", type=float, default=50.0, help="MIS slow step (first one for mis-adaptive)")
    ap.add_argument("--h-fast", type=float, default=1.0, help="fixed fast RK4 step; 0: adaptive fast ERK")
    ap.add_argument("--fast-rtol", type=float, default=1e-5)
    ap.add_argument("--checks", type=int, default=10)
    ap.add_argument("--graph", type=int, default=1, help="replay step sequences from HIP graphs")
    ap.add_argument("--pid-alt-sign", type=int, default=0,
                    help="1: PID with +k2 on the previous error (ARKODE's form) instead of the printed one")
    a = ap.parse_args(argv)

    import torch
    import synth
    from . import rtbte as R

    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    wl = synth.build(a.workload, **({} if a.L is None else {"L": a.L}))
    gen_s = time.perf_counter() - t0
    log(f"[run] {a.workload}: n_el {wl.n_el} n_ph {wl.n_ph}, generated in {gen_s:.1f} s")
    fast_kw = dict(fast_mode=1, h_fast=a.h_fast) if a.h_fast > 0 else \
        dict(fast_mode=0, fast_rtol=a.fast_rtol, fast_atol_el=a.atol_el, fast_atol_ph=a.atol_ph)
    t0 = time.perf_counter()
    ctx = R.Context(wl.problem_arrays(), precision=R.FP64 if a.precision == "fp64" else R.MIXED,
                    rtol=a.rtol, atol_el=a.atol_el, atol_ph=a.atol_ph, use_graph=a.graph,
                    pid_alt_sign=a.pid_alt_sign, **fast_kw)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    counts = ctx.counts()
    log(f"[run] context ({a.precision}) in {create_s:.1f} s, channels {counts}")

    dev = torch.device("cuda:0")
    y = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    h = torch.zeros(1, dtype=torch.float64, device=dev)
    hs = torch.full((1,), a.h_slow, dtype=torch.float64, device=dev)
    ne = wl.n_el
    modes = np.arange(wl.n_ph, dtype=np.int32) % wl.grid["n_modes"]

    def advance(tc):
        if a.method == "erk":
            ctx.step_adaptive(y, t, h, tc)
        elif a.method == "rk4":
            n = int(round((tc - float(t.item())) / a.h))
            if n > 0:
                ctx.step_rk4(y, t, a.h, n)
        elif a.method == "mis":
            ctx.step_multirate(y, t, h, tc, a.h_slow)
        else:
            ctx.step_multirate_adaptive(y, t, h, hs, tc)

    history = []
    wall = 0.0
    for k in range(1, a.checks + 1):
        tc = a.t_end * k / a.checks
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        advance(tc)
        torch.cuda.synchronize()
        wall += time.perf_counter() - w0
        yh = y.cpu().numpy()
        T = ctx.mode_temperatures(y, modes, wl.grid["n_modes"])
        st = ctx.stats()
        history.append(dict(t_fs=float(t.item()), wall_s=wall, carriers=float(yh[:ne].sum()),
                            phonon_T_K=[round(float(x), 3) for x in T], rhs_eph=st["n_rhs_eph"],
                            rhs_phph=st["n_rhs_phph"]))
        log(f"[run] t = {t.item():.1f} fs, wall {wall:.2f} s, {st['n_rhs_phph']} ph-ph / {st['n_rhs_eph']} e-ph "
            f"evaluations, branch T = {', '.join(f'{x:.1f}' for x in T)} K")
    st = ctx.stats()
    res = dict(workload=a.workload, n_el=wl.n_el, n_ph=wl.n_ph, channels=list(counts), precision=a.precision,
               method=a.method, t_end_fs=a.t_end, wall_s=wall, sim_ps_per_s=a.t_end * 1e-3 / wall,
               generate_s=gen_s, create_s=create_s, steps=st["n_accept"], rejected=st["n_reject"],
               fast_steps=st["n_fast_accept"], rhs_eph=st["n_rhs_eph"], rhs_phph=st["n_rhs_phph"],
               h_last=st["h_last"], h_slow_last=float(hs.item()) if a.method == "mis-adaptive" else None,
               options=dict(rtol=a.rtol, atol_el=a.atol_el, atol_ph=a.atol_ph, h=a.h, h_slow=a.h_slow,
                            h_fast=a.h_fast, fast_rtol=a.fast_rtol, pid_alt_sign=a.pid_alt_sign),
               history=history)
    print(json.dumps(res))
    return res


if __name__ == "__main__":
    main()
