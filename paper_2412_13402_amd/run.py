"""Run one workload from its initial state to an end time with one of the
integrators and report wall time, simulated ps per second, the work done and
the effective phonon-branch temperatures at the end.

    python -m paper_2412_13402_amd.run --workload graphene2d --method erk --t-end 10000
    python -m paper_2412_13402_amd.run --workload si3d --method mis --h-slow 50 --h-fast 1 --t-end 20000

    python -m paper_2412_13402_amd.run --workload graphene2d --batch 8 --batch-L 24 48 --method mis-adaptive --h-fast 0

Methods: erk (adaptive Zonneveld ERK on the whole right-hand side), rk4
(fixed steps --h), mis (MRI with MIS coupling, slow step --h-slow; fast part
by fixed RK4 steps --h-fast, or by the adaptive ERK with --fast-rtol when
--h-fast is 0), mis-adaptive (the same with the slow step chosen from rtol by
step doubling, starting from --h-slow).  With --batch N, N independent
instances of the workload's model (grid sides and carrier temperatures drawn
uniformly from --batch-L and --batch-T) advance together in one context:
each with its own ERK step, or on common slow steps for the multirate
methods; the history then holds one entry per instance.  Progress lines go
to stderr at --checks evenly spaced times; one JSON line goes to stdout at
the end.
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
    ap.add_argument("--L", type=int, default=None, help="grid side (default: the recipe's; --batch draws its own)")
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
    ap.add_argument("--batch", type=int, default=0, help="N > 0: a batch of N instances of the model")
    ap.add_argument("--batch-L", type=int, nargs=2, default=(24, 72), help="grid side range of a batch")
    ap.add_argument("--batch-T", type=float, nargs=2, default=(500.0, 3000.0),
                    help="initial carrier temperature range of a batch (K)")
    a = ap.parse_args(argv)

    import torch
    import synth
    from . import rtbte as R

    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    if a.batch > 0:
        wls = synth.build_batch(a.batch, tuple(a.batch_L), tuple(a.batch_T), recipe=a.workload)
    else:
        wls = [synth.build(a.workload, **({} if a.L is None else {"L": a.L}))]
    gen_s = time.perf_counter() - t0
    n = len(wls)
    log(f"[run] {a.workload} x {n}: n_el {[w.n_el for w in wls]} n_ph {[w.n_ph for w in wls]}, "
        f"generated in {gen_s:.1f} s")
    fast_kw = dict(fast_mode=1, h_fast=a.h_fast) if a.h_fast > 0 else \
        dict(fast_mode=0, fast_rtol=a.fast_rtol, fast_atol_el=a.atol_el, fast_atol_ph=a.atol_ph)
    t0 = time.perf_counter()
    ctx = R.Context([w.problem_arrays() for w in wls], precision=R.FP64 if a.precision == "fp64" else R.MIXED,
                    rtol=a.rtol, atol_el=a.atol_el, atol_ph=a.atol_ph, use_graph=a.graph,
                    pid_alt_sign=a.pid_alt_sign, **fast_kw)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    counts = [list(ctx.counts(i)) for i in range(n)]
    log(f"[run] context ({a.precision}) in {create_s:.1f} s, channels {[sum(c) for c in counts]}")

    dev = torch.device("cuda:0")
    y = torch.tensor(np.concatenate([w.y0 for w in wls]), dtype=torch.float64, device=dev)
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    hs = torch.full((n,), a.h_slow, dtype=torch.float64, device=dev)
    layout = [ctx.layout(i) for i in range(n)]
    modes = [np.arange(w.n_ph, dtype=np.int32) % w.grid["n_modes"] for w in wls]

    def advance(tc):
        if a.method == "erk":
            ctx.step_adaptive(y, t, h, tc)
        elif a.method == "rk4":
            k = int(round((tc - float(t[0].item())) / a.h))
            if k > 0:
                ctx.step_rk4(y, t, a.h, k)
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
        th = t.cpu().numpy()
        entry = []
        for i, (w, (off, ne, nph)) in enumerate(zip(wls, layout)):
            T = ctx.mode_temperatures(y, modes[i], w.grid["n_modes"], inst=i)
            st = ctx.stats(i)
            entry.append(dict(t_fs=float(th[i]), carriers=float(yh[off:off + ne].sum()),
                              phonon_T_K=[round(float(x), 3) for x in T], rhs_eph=st["n_rhs_eph"],
                              rhs_phph=st["n_rhs_phph"]))
        e0 = dict(entry[0], wall_s=wall)
        history.append(e0 if n == 1 else dict(wall_s=wall, instances=entry))
        log(f"[run] t = {th[0]:.1f} fs, wall {wall:.2f} s, instance 0: {e0['rhs_phph']} ph-ph / "
            f"{e0['rhs_eph']} e-ph evaluations, branch T = {', '.join(f'{x:.1f}' for x in e0['phonon_T_K'])} K")
    sts = [ctx.stats(i) for i in range(n)]
    one = lambda key: sts[0][key] if n == 1 else [s_[key] for s_ in sts]
    res = dict(workload=a.workload, n_inst=n, n_el=one_or([w.n_el for w in wls]), n_ph=one_or([w.n_ph for w in wls]),
               channels=counts[0] if n == 1 else counts, precision=a.precision, method=a.method,
               t_end_fs=a.t_end, wall_s=wall, sim_ps_per_s=n * a.t_end * 1e-3 / wall,
               generate_s=gen_s, create_s=create_s, steps=one("n_accept"), rejected=one("n_reject"),
               fast_steps=one("n_fast_accept"), rhs_eph=one("n_rhs_eph"), rhs_phph=one("n_rhs_phph"),
               h_last=one("h_last"), h_slow_last=float(hs[0].item()) if a.method == "mis-adaptive" else None,
               health=one("health"),
               options=dict(rtol=a.rtol, atol_el=a.atol_el, atol_ph=a.atol_ph, h=a.h, h_slow=a.h_slow,
                            h_fast=a.h_fast, fast_rtol=a.fast_rtol, pid_alt_sign=a.pid_alt_sign,
                            batch=a.batch, batch_L=list(a.batch_L), batch_T=list(a.batch_T)),
               history=history)
    print(json.dumps(res))
    return res


def one_or(v):
    return v[0] if len(v) == 1 else v


if __name__ == "__main__":
    main()
