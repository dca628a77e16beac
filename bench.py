"""Benchmark of the rt-BTE hot path on one MI355X.

Workload: the graphene-like coupled e-ph + ph-ph problem (120x120 k = q grid,
2 pi bands, 6 phonon branches, ~1.6e8 + 0.8e8 e-ph and ~5e8 ph-ph channels,
6.1e8 stored), advanced by the adaptive Zonneveld ERK (rtol 1e-6).  One
benchmark step is one accepted ERK step: its attempts (5 right-hand-side
evaluations each, every stored channel streamed once per evaluation), the
fused stage updates, the WRMS error norm and the device-side PID control.

Prints one JSON line:
* value: stored channels per second over whole ERK steps (channels streamed
  per right-hand side times right-hand sides per second; the rate over the
  channels the sums contain, which counts each folded ph-ph emission pair
  twice, is value_summed_channels);
* roofline: the collision kernel's algorithmic bytes per launch over its
  HIP-event-timed duration, against the 8 TB/s HBM peak;
* cpu_baseline: the FP64 oracle on this host's cores, same basis (and the
  simulated ps/s it would reach on the horizon run, extrapolated from its
  right-hand-side time);
* horizon: simulated ps per second from the initial state to 1 ps, FP64 and
  mixed, printed and ARKODE PID forms, each with its end-time error against
  an FP64 reference at rtol 1e-9 (the top-level sim_ps_per_s is the FP64
  printed-form figure);
* fp64_plain_channels, mixed: the same steps with the plain 16-byte FP64
  channels and in mixed precision (speedup, kernel roofline, RHS error per
  step against the oracle, populations after 1 ps of RK4 against FP64);
* batched: 64 graphene-like instances in one autotuned, graph-replayed mixed
  context against the same instances one by one in FP64, with errors against
  an FP64 reference, the mixed-vs-FP64 population error on fixed steps, and
  the oracle's right-hand side on a sample of the instances;
* si3d: the silicon-like 40^3 workload, MIS against the adaptive ERK, slow
  and fast right-hand-side rooflines, the oracle on a row sample;
* toy: the small e-ph-only RK4 case beside the oracle.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the collision kernels' source (comments and blank lines left
    out, so that the hash changes with the code only)."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2412_13402_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(workload, precision):
    """HBM bytes per launch of the collision kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(precision)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


TRAFFIC_LEGS = (("fp64", "k_items", ("roofline",)),
                ("fp64_plain", "k_items", ("fp64_plain_channels", "roofline")),
                ("mixed", "k_items_mixed", ("mixed", "roofline")))


def _counter_means(path, counter):
    """Per-kernel mean of one rocprofv3 counter (KiB per dispatch), and its
    reading for the run's first copy kernel (the 1 GiB device-to-device copy
    of --calibrate-copy, the first copy the benchmark makes), from a `--pmc`
    run's CSV output."""
    import csv
    import glob
    acc, copy = {}, (None, 0.0)
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                name, v = row["Kernel_Name"], float(row["Counter_Value"])
                if "copyBuffer" in name:
                    d = int(row["Dispatch_Id"])
                    if copy[0] is None or d < copy[0]:
                        copy = (d, v)
                acc.setdefault(name.split("(")[0], []).append(v)
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}, copy[1]


def _template_args(name):
    return [a.strip() for a in name[name.index("<") + 1:name.rindex(">")].split(",")]


def traffic_summary(fetch_dir, write_dir, bench_json, workload, out_path=None):
    """Write profiles/traffic_<workload>.json from two rocprofv3 `--pmc` runs
    of this benchmark with `--calibrate-copy` (FETCH_SIZE, then WRITE_SIZE)
    and the JSON line the first run printed: HBM bytes per launch of each
    collision kernel, each counter scaled by what it reads for the 1 GiB
    device-to-device copy, beside the algorithmic bytes per launch."""
    fetch, fcopy = _counter_means(fetch_dir, "FETCH_SIZE")
    write, wcopy = _counter_means(write_dir, "WRITE_SIZE")
    with open(bench_json) as f:
        rec = json.loads(f.read().strip().splitlines()[-1])
    gib = float(1 << 30)
    fs, ws = gib / (fcopy * 1024), gib / (wcopy * 1024)
    legs = ("--steps 2 --warmup 1 --no-cpu-baseline --no-errors --no-batched --no-toy --no-si3d --no-horizon "
            "--no-matrix-free --calibrate-copy")
    out = {"workload": rec["config"]["workload"],
           "commands": [f"cd /tmp && rocprofv3 --pmc {c} -d <out>/{d} -o bench --output-format csv -- "
                        f"python3 <repo>/bench.py {legs} > <out>/{d}.json" for c, d in
                        (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))] +
                       ["python3 <repo>/bench.py --traffic-summary <out>/fetch <out>/write <out>/fetch.json"],
           "copy_reference": {"bytes_read": gib, "bytes_written": gib, "fetch_kib_raw": fcopy,
                              "write_kib_raw": wcopy},
           "fetch_scale": fs, "write_scale": ws}
    for leg, base, keys in TRAFFIC_LEGS:
        r = rec
        for k in keys:
            r = r.get(k) if r else None
        if not r:
            continue
        pack = leg != "fp64_plain"
        pick = [n for n in fetch if n.split("<")[0].endswith("::" + base)
                and _template_args(n)[1] == ("true" if pack else "false")
                and all(a == "false" for a in _template_args(n)[2:])]
        if len(pick) != 1 or pick[0] not in write:
            continue
        n = pick[0]
        hbm = (fetch[n][1] * fs + write[n][1] * ws) * 1024
        out[leg] = {"kernel": n, "kernel_source_hash": kernel_source_hash(), "dispatches": fetch[n][0],
                    "fetch_kib_per_dispatch_raw": fetch[n][1], "write_kib_per_dispatch_raw": write[n][1],
                    "hbm_bytes_per_launch": hbm,
                    "algorithmic_bytes_per_launch": r["algorithmic_bytes_per_launch"],
                    "ratio": hbm / r["algorithmic_bytes_per_launch"]}
    path = out_path or os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({k: v.get("ratio") for k, v in out.items() if isinstance(v, dict) and "ratio" in v}))


def fp64_dtype(ctx):
    """The arithmetic type of the FP64 path, with the storage rounding of its
    channel weights named when the layout rounds them."""
    _, nbytes, u = ctx.weight_format()
    if u > 0:
        import math
        return (f"f64 (channel weights stored in {nbytes}-byte packed channels to 2^{math.log2(u):.0f} "
                f"relative; arithmetic, state and control FP64)")
    return "f64"


def cpu_baseline(wl, seconds, stored):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    whole Zonneveld ERK attempts (5 full right-hand sides each).  Its rate is
    stated on the same basis as the GPU's: right-hand sides per second times
    the stored channels of one right-hand side (`stored`)."""
    import numpy as np
    from __graft_entry__ import _ensure_built
    _ensure_built(need_oracle=True)
    import oracle
    from oracle import integrators as I
    t0 = time.perf_counter()
    o = oracle.Oracle(wl.problem_arrays())
    build_s = time.perf_counter() - t0
    ch = sum(o.counts())
    n = 0
    y = wl.y0.copy()
    t0 = time.perf_counter()
    while True:
        ynew, lte = I.erk_attempt(o.rhs, y, 0.5)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    assert np.all(np.isfinite(ynew))
    cores = oracle.threads()
    # one thread: a single full right-hand side of the same state
    oracle.set_threads(1)
    t1 = time.perf_counter()
    o.rhs(y)
    el1 = time.perf_counter() - t1
    oracle.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return o, dict(value=n * 5 * stored / el, unit="channels/s", cores=cores, kind="oracle",
                   sample=f"{n} Zonneveld ERK attempt(s) = {5 * n} full right-hand sides of the "
                          f"same workload from its initial state ({el:.1f} s; list build {build_s:.1f} s "
                          f"untimed); rate in stored channels per right-hand side ({stored}), as the GPU value",
                   value_summed_channels=n * 5 * ch / el,
                   one_thread_value=stored / el1, one_thread_sample=f"1 full right-hand side ({el1:.1f} s)",
                   cpu_model=model)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="graphene2d")
    ap.add_argument("--L", type=int, default=None, help="grid side override (smaller test runs)")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--group-rows-el", type=int, default=0, help="electron rows per group (0: library choice)")
    ap.add_argument("--group-rows-ph", type=int, default=0, help="phonon rows per group (0: library choice)")
    ap.add_argument("--item-channels", type=int, default=0, help="channels per work item (0: library choice)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--err-steps", type=int, default=5, help="mixed steps with a per-step RHS error report")
    ap.add_argument("--no-errors", action="store_true", help="skip the mixed accuracy pass (profiling runs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 leg with plain 16-byte channels")
    ap.add_argument("--batch", type=int, default=64, help="instances of the batched leg")
    ap.add_argument("--batch-t-end", type=float, default=200.0, help="simulated fs of the batched leg")
    ap.add_argument("--no-si3d", action="store_true",
                    help="skip the silicon-like 3D leg (40^3, ~2.5e9 channels): MIS vs ERK")
    ap.add_argument("--no-toy", action="store_true", help="skip the small RK4 leg")
    ap.add_argument("--si-L", type=int, default=40)
    ap.add_argument("--si-t-end", type=float, default=200.0)
    ap.add_argument("--si-sample-rows", type=int, default=40000,
                    help="rows of the silicon-like workload the oracle baseline evaluates")
    ap.add_argument("--no-horizon", action="store_true",
                    help="skip the runs from the initial state to --horizon-fs (simulated ps/s at a stated error)")
    ap.add_argument("--horizon-fs", type=float, default=1000.0)
    ap.add_argument("--ref-rtol", type=float, default=1e-9,
                    help="relative tolerance of the FP64 reference runs the end-time errors are taken against")
    ap.add_argument("--batch-rk4-fs", type=float, default=1000.0,
                    help="batched leg: fixed-step RK4 span of the mixed-vs-FP64 population check")
    ap.add_argument("--batch-rk4-h", type=float, default=2.0,
                    help="fixed RK4 step (fs) of the batched precision check: below RK4's stability limit "
                         "of every instance (2.9 fs for the stiffest of the 64 at its initial state)")
    ap.add_argument("--no-tune", action="store_true", help="batched leg: default launch shape, no autotuning")
    ap.add_argument("--no-matrix-free", action="store_true",
                    help="skip the matrix-free ph-ph weights leg (|V3|^2 model evaluated in the kernel)")
    ap.add_argument("--tiled", type=int, default=0, choices=(0, 1),
                    help="0 (default): per-item collision kernels; 1: tiled (partners staged in LDS)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a known-size reference for HBM counters)")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "BENCH_JSON"),
                    help="no run: write profiles/traffic_<workload>.json from two rocprofv3 --pmc runs "
                         "(FETCH_SIZE, WRITE_SIZE) of this benchmark with --calibrate-copy")
    ap.add_argument("--valu-summary", nargs=2, metavar=("PMC_DIR", "BENCH_JSON"),
                    help="no run: write profiles/valu_matrix_free_<workload>.json from a rocprofv3 --pmc "
                         "SQ_INSTS_VALU run of this benchmark (" + MF_VALU_LEGS + ")")
    args = ap.parse_args()
    if args.valu_summary:
        valu_summary(*args.valu_summary, args.workload if args.L is None else f"{args.workload}_L{args.L}")
        return
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary, args.workload if args.L is None else f"{args.workload}_L{args.L}")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row sharding is a design, not a build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_2412_13402_amd as P
    from __graft_entry__ import _ensure_built
    _ensure_built()

    if args.calibrate_copy:
        src = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    over = {} if args.L is None else {"L": args.L}
    t0 = time.perf_counter()
    wl = synth.build(args.workload, **over)
    gen_s = time.perf_counter() - t0
    log(f"[bench] workload {args.workload}: n_el={wl.n_el} n_ph={wl.n_ph} entries "
        f"{len(wl.eph_row)} e-ph + {len(wl.pp_row)} ph-ph, generated in {gen_s:.1f} s")
    t0 = time.perf_counter()
    ctx = P.Context(wl.problem_arrays(), rtol=args.rtol, atol_el=1e-9, atol_ph=1e-12,
                    group_rows_el=args.group_rows_el, group_rows_ph=args.group_rows_ph,
                    item_channels=args.item_channels, tiled=args.tiled)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    counts = ctx.counts()
    C = sum(counts)
    stored = ctx.stored_counts()
    CS = sum(stored)
    log(f"[bench] create {create_s:.1f} s; channels e-ph {counts[0]}, ph-e {counts[1]}, "
        f"ph-ph {counts[2]} (total {C}; stored {CS}); rows per group (el, ph), channels per item {ctx.tuning()}")
    leg = timed_steps(ctx, wl, args, CS, "fp64")
    k = leg["kernel"]
    traffic = measured_traffic(args.workload if args.L is None else f"{args.workload}_L{args.L}", "fp64")
    rec = {
        "metric": "RHS scattering channels/s & % HBM peak; simulated ps/s at fixed error",
        "value": leg["value"],
        "unit": "channels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": fp64_dtype(ctx),
        "data": "synthetic (seeded graphene-like band/phonon model and channel lists; no first-principles data)",
        "config": {
            "workload": f"{args.workload}: {'x'.join([str(wl.grid['L'])] * 2)} k=q grid, 2 bands, 6 branches, "
                        f"FP64, adaptive Zonneveld ERK rtol {args.rtol:g}",
            "channels_eph": counts[0], "channels_phe": counts[1], "channels_phph": counts[2],
            "stored_channels": list(stored),
            "value_counts": "stored channels (streamed once per right-hand side) x right-hand sides / s",
            "n_y": wl.n_y, "rhs_per_step": leg["rhs_per_step"],
            "rows_per_group_el": ctx.tuning()[0], "rows_per_group_ph": ctx.tuning()[1],
            "channels_per_item": ctx.tuning()[2],
        },
        "value_summed_channels": leg["value"] * C / CS,
        "sim_ps_per_s": leg["sim_ps_per_s"],
        "sim_ps_per_s_note": f"the {args.steps} timed steps ({leg['t_span'][0]:.1f} -> {leg['t_span'][1]:.1f} fs); "
                             "the same at a stated error from the initial state: horizon",
        "hbm_frac": k["achieved"] / HBM_PEAK_GBS,
        "roofline": dict(k, traffic=traffic),
        "create_s": create_s,
        "generate_s": gen_s,
    }
    fmt = ctx.weight_format()
    rec["config"]["fp64_channel_bytes"] = fmt[1]
    rec["config"]["fp64_weight_rounding"] = fmt[2]
    rec["roofline"]["launch_spread"] = launch_spread(ctx, torch, leg["y"])
    rec["achievable"] = achievable_bandwidth(torch)

    if not args.no_plain:
        # the same steps with the plain 16-byte FP64 channels (two 32-bit
        # indices and the full FP64 weight), for comparison
        t0 = time.perf_counter()
        ctx_p = P.Context(wl.problem_arrays(), rtol=args.rtol, atol_el=1e-9, atol_ph=1e-12,
                          group_rows_el=args.group_rows_el, group_rows_ph=args.group_rows_ph,
                          item_channels=args.item_channels, fp64_layout=P.rtbte.F64_PLAIN)
        torch.cuda.synchronize()
        cp = time.perf_counter() - t0
        leg_p = timed_steps(ctx_p, wl, args, CS, "fp64 plain", start=leg["start"])
        rec["fp64_plain_channels"] = {
            "value": leg_p["value"], "unit": "channels/s", "ms_per_step": leg_p["ms_per_step"],
            "sim_ps_per_s": leg_p["sim_ps_per_s"], "channel_bytes": 16,
            "roofline": dict(leg_p["kernel"], traffic=measured_traffic(
                args.workload if args.L is None else f"{args.workload}_L{args.L}", "fp64_plain")),
            "create_s": cp,
        }
        del ctx_p

    ctx_m = None
    if not args.no_mixed:
        t0 = time.perf_counter()
        ctx_m = P.Context(wl.problem_arrays(), precision=P.rtbte.MIXED, rtol=args.rtol, atol_el=1e-9,
                          atol_ph=1e-12, group_rows_el=args.group_rows_el, group_rows_ph=args.group_rows_ph,
                          item_channels=args.item_channels, tiled=args.tiled)
        torch.cuda.synchronize()
        create_m = time.perf_counter() - t0
        leg_m = timed_steps(ctx_m, wl, args, CS, "mixed", start=leg["start"])
        km = leg_m["kernel"]
        tm = measured_traffic(args.workload if args.L is None else f"{args.workload}_L{args.L}", "mixed")
        rec["mixed"] = {
            "value": leg_m["value"], "unit": "channels/s", "ms_per_step": leg_m["ms_per_step"],
            "sim_ps_per_s": leg_m["sim_ps_per_s"],
            "speedup_sim_ps_per_s_vs_fp64": leg_m["sim_ps_per_s"] / leg["sim_ps_per_s"],
            "speedup_rhs_kernel_vs_fp64": k["avg_launch_ms"] / km["avg_launch_ms"],
            "rhs_per_step": leg_m["rhs_per_step"],
            "t_span_fs": leg_m["t_span"], "fp64_t_span_fs": leg["t_span"],
            "dtype": f"weights in {ctx_m.weight_format()[1]}-byte packed channels (relative rounding "
                     f"{ctx_m.weight_format()[2]:.2g}) with per-512 FP32 scales; FP32 population codes, "
                     "products and compensated lane sums; FP64 state, stages, WRMS and control",
            "roofline": dict(km, traffic=tm, launch_spread=launch_spread(ctx_m, torch, leg_m["y"])),
            "create_s": create_m,
        }

    o = None
    if not args.no_cpu_baseline:
        log("[bench] oracle baseline on host cores ...")
        o, cb = cpu_baseline(wl, args.cpu_seconds, CS)
        rec["cpu_baseline"] = cb
        # parity of the GPU right-hand side at the final state, every row
        yf = leg["y"].cpu().numpy()
        out = torch.empty_like(leg["y"])
        ctx.rhs(leg["y"], out, P.PART_ALL)
        torch.cuda.synchronize()
        ref, S, A = o.rhs(yf, scales=True)
        g = out.cpu().numpy()
        rec["rhs_err_vs_oracle"] = {
            "max_row_err_over_magnitude": float(np.max(np.abs(g - ref) / np.maximum(A, 1e-300))),
            "normwise": float(np.linalg.norm(g - ref) / np.linalg.norm(ref)),
        }
    if ctx_m is not None and not args.no_errors:
        rec["mixed"].update(mixed_errors(P, torch, np, ctx, ctx_m, wl, o, args))
    if not args.no_matrix_free:
        rec["matrix_free_pp"] = matrix_free_leg(P, torch, np, wl, args, ctx, o)
    if not args.no_horizon:
        hz = horizon_leg(P, torch, np, wl, args, ctx, ctx_m)
        rec["horizon"] = hz
        rec["sim_ps_per_s"] = hz["fp64"]["sim_ps_per_s"]
        rec["sim_ps_per_s_note"] = (f"FP64 adaptive ERK (printed PID form) from the initial state to "
                                    f"{args.horizon_fs:g} fs, end-time error vs an FP64 run at rtol "
                                    f"{args.ref_rtol:g}: carriers {hz['fp64']['err_carriers']:.2e}, phonons "
                                    f"{hz['fp64']['err_phonons']:.2e} (horizon)")
        if "cpu_baseline" in rec:
            # the oracle on the same run, extrapolated from its right-hand-side time
            s_rhs = CS / rec["cpu_baseline"]["value"]
            n_rhs = 5 * (hz["fp64"]["accepted"] + hz["fp64"]["rejected"])
            rec["cpu_baseline"]["sim_ps_per_s_extrapolated"] = args.horizon_fs * 1e-3 / (n_rhs * s_rhs)
            rec["cpu_baseline"]["sim_ps_per_s_note"] = (
                f"extrapolated, not run: the FP64 run to {args.horizon_fs:g} fs takes {n_rhs} right-hand sides "
                f"(5 per attempt), at the oracle's {s_rhs:.3f} s each")
    del ctx, ctx_m, o, leg
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if not args.no_batched:
        rec["batched"] = batched_leg(P, torch, np, args)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if not args.no_si3d:
        rec["si3d"] = si3d_leg(P, torch, np, args)
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    if not args.no_toy:
        rec["toy"] = toy_leg(P, torch, np, with_oracle=not args.no_cpu_baseline)
    print(json.dumps(rec), flush=True)


VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9      # CUs x SIMDs x lanes x clock
MF_VALU_LEGS = "--no-batched --no-si3d --no-horizon --no-toy --no-cpu-baseline --no-errors --no-plain --no-mixed " \
               "--steps 2 --warmup 1"


def valu_summary(pmc_dir, bench_json, workload, out_path=None):
    """Write profiles/valu_matrix_free_<workload>.json from a rocprofv3
    `--pmc SQ_INSTS_VALU` run of this benchmark (MF_VALU_LEGS) and the JSON
    line it printed: VALU lane-instructions per stored ph-ph channel of the
    matrix-free FP64 collision kernel, from its ph-ph-only launches (the
    dispatches with the fewest instructions; the whole-RHS launches also
    carry the e-ph and ph-e work)."""
    import csv
    import glob
    vals = []
    name = None
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                n = row["Kernel_Name"].split("(")[0]
                if row["Counter_Name"] != "SQ_INSTS_VALU" or not n.split("<")[0].endswith("::k_items"):
                    continue
                if _template_args(n)[1:] == ["true", "false", "true"]:   # packed FP64, matrix-free
                    vals.append(float(row["Counter_Value"]))
                    name = n
    with open(bench_json) as f:
        rec = json.loads(f.read().strip().splitlines()[-1])
    stored_pp = rec["config"]["stored_channels"][2]
    v = min(vals)
    out = {"workload": rec["config"]["workload"],
           "commands": [f"cd /tmp && rocprofv3 --pmc SQ_INSTS_VALU -d <out>/valu -o valu --output-format csv -- "
                        f"python3 <repo>/bench.py {MF_VALU_LEGS} > <out>/valu.json",
                        "python3 <repo>/bench.py --valu-summary <out>/valu <out>/valu.json"],
           "kernel": name, "kernel_source_hash": kernel_source_hash(), "dispatches": len(vals),
           "valu_wave_instructions_phph_launch": v, "stored_phph_channels": stored_pp,
           "lane_instructions_per_channel": v * 64 / stored_pp}
    path = out_path or os.path.join(ROOT, "profiles", f"valu_matrix_free_{workload}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({"lane_instructions_per_channel": out["lane_instructions_per_channel"]}))


def measured_mf_valu(workload):
    """VALU lane-instructions per ph-ph channel of the matrix-free kernel from
    the committed counter summary, if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", f"valu_matrix_free_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d["lane_instructions_per_channel"] if d.get("kernel_source_hash") == kernel_source_hash() else None


def matrix_free_leg(P, torch, np, wl, args, ctx64, o):
    """Matrix-free ph-ph weights: the ph-ph channels keep partners and flags
    only, and every right-hand side recomputes prefactor * |V3|^2 * delta from
    the generator's |V3|^2 model (Philox4x32-10 over the canonical triplet,
    Box-Muller, lognormal) in FP64.  Times the ph-ph part and the whole
    right-hand side against the stored-weight FP64 context, and checks the
    matrix-free right-hand side against the oracle at the initial state."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    res = {"what": "ph-ph weights recomputed from the |V3|^2 model at every right-hand side (FP64); "
                   "e-ph and ph-e from stored weights"}
    y = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    for name, kw in (("fp64", {}), ("mixed", dict(precision=P.rtbte.MIXED))):
        c = P.Context(dict(wl.problem_arrays(), pp_v2=None), pp_model=wl.pp_model(), **kw)
        torch.cuda.synchronize()
        leg = {"create_s": time.perf_counter() - t0}
        for part, label in ((P.PART_PHPH, "phph"), (P.PART_ALL, "all")):
            r = kernel_roofline(c, torch, y, part)
            leg[f"{label}_ms"] = r["avg_launch_ms"]
            leg[f"{label}_bytes_per_launch"] = r["algorithmic_bytes_per_launch"]
        stored = c.stored_counts()
        leg["phph_channels_per_s"] = stored[2] / (leg["phph_ms"] * 1e-3)
        if name == "fp64":
            ref = kernel_roofline(ctx64, torch, y, P.PART_PHPH)
            leg["stored_weights_phph_ms"] = ref["avg_launch_ms"]
            leg["slowdown_vs_stored"] = leg["phph_ms"] / ref["avg_launch_ms"]
            ipc = measured_mf_valu(args.workload if args.L is None else f"{args.workload}_L{args.L}")
            leg["roofline"] = None
            if ipc:
                ach = ipc * stored[2] / (leg["phph_ms"] * 1e-3)
                leg["roofline"] = {"bound": "alu", "achieved": ach / 1e12, "peak": VALU_PEAK_LANE_OPS / 1e12,
                                   "unit": "T VALU lane-instructions/s", "frac": ach / VALU_PEAK_LANE_OPS,
                                   "instructions_per_channel": ipc}
            if o is not None:
                out = torch.empty_like(y)
                c.rhs(y, out, P.PART_ALL)
                torch.cuda.synchronize()
                g = out.cpu().numpy()
                rf, S, A = o.rhs(wl.y0, scales=True)
                leg["rhs_err_vs_oracle"] = {
                    "max_row_err_over_magnitude": float(np.max(np.abs(g - rf) / np.maximum(A, 1e-300))),
                    "normwise": float(np.linalg.norm(g - rf) / np.linalg.norm(rf))}
        res[name] = leg
        log(f"[bench] matrix-free {name}: ph-ph {leg['phph_ms']:.3f} ms, whole RHS {leg['all_ms']:.3f} ms")
        del c
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
    return res


def horizon_leg(P, torch, np, wl, args, ctx64, ctx_m):
    """Simulated ps per wall second at a stated error (Methods, choice of
    tolerances and reference solutions): each configuration advances the
    workload from its initial state to the horizon with the adaptive ERK (the
    benchmark's rtol; h = 0 asks for the starting-step estimate), and its end
    state is compared with an FP64 reference run at a tighter tolerance,
    ||x - x_ref|| / ||x_ref|| over the carriers and over the phonons.
    Configurations: FP64 and mixed precision, each with the printed PID form
    (the default) and with ARKODE's (+k2 on eps_{k-1})."""
    dev = torch.device("cuda:0")
    T = args.horizon_fs
    probs = wl.problem_arrays()
    y0 = torch.tensor(wl.y0, dtype=torch.float64, device=dev)

    def run(ctx):
        y = y0.clone()
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        h = torch.zeros(1, dtype=torch.float64, device=dev)
        ctx.reset()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ctx.step_adaptive(y, t, h, T)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        st = ctx.stats()
        assert t.item() == T
        return y.cpu().numpy(), wall, st

    t0 = time.perf_counter()
    ref_tol = dict(rtol=args.ref_rtol, atol_el=1e-12, atol_ph=1e-15)
    ctx_r = P.Context(probs, **ref_tol)
    yref, wref, sref = run(ctx_r)
    del ctx_r
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    ne = wl.n_el
    nrm = np.linalg.norm
    res = {"horizon_fs": T, "rtol": args.rtol, "atol_el": 1e-9, "atol_ph": 1e-12,
           "reference": dict(ref_tol, accepted=sref["n_accept"], rejected=sref["n_reject"], wall_s=wref,
                             note="FP64 adaptive ERK, printed PID form")}
    log(f"[bench] horizon reference (rtol {args.ref_rtol:g}): {T:g} fs in {wref:.2f} s, "
        f"{sref['n_accept']} steps")
    tol = dict(rtol=args.rtol, atol_el=1e-9, atol_ph=1e-12)
    cases = [("fp64", ctx64, None), ("fp64_arkode_pid", None, dict(precision=P.rtbte.FP64, pid_alt_sign=1))]
    if ctx_m is not None:
        cases += [("mixed", ctx_m, None), ("mixed_arkode_pid", None, dict(precision=P.rtbte.MIXED, pid_alt_sign=1))]
    for name, ctx, kw in cases:
        own = ctx is None
        if own:
            ctx = P.Context(probs, **tol, **kw)
            yw = y0.clone()
            tw = torch.zeros(1, dtype=torch.float64, device=dev)
            hw_ = torch.zeros(1, dtype=torch.float64, device=dev)
            ctx.step_adaptive(yw, tw, hw_, 20.0)     # warm-up (first launches)
            del yw
        y, wall, st = run(ctx)
        res[name] = {"wall_s": wall, "sim_ps_per_s": T * 1e-3 / wall, "accepted": st["n_accept"],
                     "rejected": st["n_reject"],
                     "err_carriers": float(nrm(y[:ne] - yref[:ne]) / nrm(yref[:ne])),
                     "err_phonons": float(nrm(y[ne:] - yref[ne:]) / nrm(yref[ne:]))}
        log(f"[bench] horizon {name}: {T:g} fs in {wall:.2f} s ({st['n_accept']} accepted, {st['n_reject']} "
            f"rejected), errors {res[name]['err_carriers']:.2e} / {res[name]['err_phonons']:.2e}")
        if own:
            del ctx
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    res["speedup_mixed_vs_fp64"] = res["fp64"]["wall_s"] / res["mixed"]["wall_s"] if "mixed" in res else None
    res["total_s"] = time.perf_counter() - t0
    return res


def toy_leg(P, torch, np, with_oracle=True):
    """The small e-ph-only case (18x18 square grid, 3 modes): fixed-step RK4,
    1 fs x 100, on the GPU (steps replayed from HIP graphs) and, beside it,
    the same run of the oracle on the host cores; launch-bound on the GPU, so
    no roofline figure."""
    import synth
    wl = synth.build("toy2d")
    ctx = P.Context(wl.problem_arrays(), use_graph=1)
    dev = torch.device("cuda:0")
    y = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    ctx.step_rk4(y, t, 1.0, 8)                  # warm-up: first launches, graph capture
    y.copy_(torch.tensor(wl.y0, dtype=torch.float64, device=dev))
    t.zero_()
    ctx.reset()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ctx.step_rk4(y, t, 1.0, 100)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    C = sum(ctx.counts())
    res = {"workload": "toy2d: 18x18 square grid, 2 bands, 3 modes, e-ph only; RK4 1 fs x 100",
           "channels": C, "gpu_wall_s": wall, "gpu_sim_ps_per_s": 0.1 / wall,
           "gpu_channels_per_s": 400 * C / wall}
    if with_oracle:                               # the CPU baseline of this case
        from __graft_entry__ import _ensure_built
        _ensure_built(need_oracle=True)
        import oracle
        from oracle import integrators as I
        o = oracle.Oracle(wl.problem_arrays())
        yr = wl.y0.copy()
        w0 = time.perf_counter()
        for _ in range(100):
            yr = I.rk4_step(o.rhs, yr, 1.0)
        ow = time.perf_counter() - w0
        res.update(oracle_wall_s=ow, oracle_sim_ps_per_s=0.1 / ow, oracle_cores=oracle.threads(),
                   max_abs_diff_vs_oracle=float(np.max(np.abs(y.cpu().numpy() - yr))))
    log(f"[bench] toy RK4 1 fs x 100: GPU {wall * 1e3:.1f} ms" +
        (f", oracle {res['oracle_wall_s'] * 1e3:.1f} ms, max |diff| {res['max_abs_diff_vs_oracle']:.2e}"
         if with_oracle else ""))
    return res


def launch_spread(ctx, torch, y, reps=20):
    """Per-launch times of the collision kernel (HIP events on its stream)
    over `reps` full right-hand sides: median, p10 and p90 in ms."""
    import numpy as np
    out = torch.empty_like(y)
    ms = []
    for _ in range(reps):
        ctx.profile(True)
        ctx.rhs(y, out, 7)
        k_ms, k_n, _ = ctx.profile_read()
        ms.append(k_ms / max(k_n, 1))
    ctx.profile(False)
    return {"reps": reps, "median_ms": float(np.median(ms)), "p10_ms": float(np.percentile(ms, 10)),
            "p90_ms": float(np.percentile(ms, 90))}


def achievable_bandwidth(torch, gib=4):
    """What plain library kernels reach on this GPU: a read-only reduction
    and a device copy over `gib` GiB (the ceiling a streaming kernel can
    expect in practice, beside the 8 TB/s peak)."""
    x = torch.ones((gib << 30) // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    res = {}
    for name, fn, nbytes in (("read_sum", lambda: x.sum(), x.numel() * 8),
                             ("copy", lambda: y.copy_(x), 2 * x.numel() * 8)):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_GBps"] = nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return res


def kernel_roofline(ctx, torch, y, parts, reps=3):
    out = torch.empty_like(y)
    ctx.rhs(y, out, parts)      # untimed
    ctx.profile(True)
    for _ in range(reps):
        ctx.rhs(y, out, parts)
    k_ms, k_n, k_bytes = ctx.profile_read()
    ctx.profile(False)
    ms = k_ms / max(k_n, 1)
    by = k_bytes / max(k_n, 1)
    ach = by / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "avg_launch_ms": ms, "algorithmic_bytes_per_launch": by}


def si3d_leg(P, torch, np, args):
    """Silicon-like 3D bulk (4 conduction bands, 6 branches): the third-order
    MIS multirate method (slow ph-ph steps of 50 fs, fixed 1 fs RK4 steps for
    the fast e-ph part) against the adaptive ERK on the whole right-hand side,
    both from the initial state to the same end time, in FP64; MIS also in
    mixed precision."""
    import synth
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    wl = synth.build("si3d", L=args.si_L)
    gen_s = time.perf_counter() - t0
    log(f"[bench] si3d {args.si_L}^3: n_el {wl.n_el} n_ph {wl.n_ph} entries {len(wl.eph_row)} e-ph + "
        f"{len(wl.pp_row)} ph-ph, generated in {gen_s:.1f} s")
    res = {"workload": f"si3d: {args.si_L}^3 k = q grid, 4 conduction bands, 6 branches, from the initial "
                       f"state to {args.si_t_end:g} fs",
           "generate_s": gen_s}
    y0 = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    hs, hf = 50.0, 1.0
    for prec, name in ((P.rtbte.FP64, "fp64"), (P.rtbte.MIXED, "mixed")):
        t0 = time.perf_counter()
        ctx = P.Context(wl.problem_arrays(), precision=prec, rtol=args.rtol, atol_el=1e-9, atol_ph=1e-12,
                        fast_mode=1, h_fast=hf)
        torch.cuda.synchronize()
        cs = time.perf_counter() - t0
        counts = ctx.counts()
        log(f"[bench] si3d {name}: create {cs:.1f} s, channels {counts}")
        leg = {"create_s": cs, "channels_eph": counts[0], "channels_phe": counts[1], "channels_phph": counts[2],
               "roofline_slow_rhs": kernel_roofline(ctx, torch, y0, P.PART_PHPH),
               "roofline_fast_rhs": kernel_roofline(ctx, torch, y0, P.PART_EPH | P.PART_PHE)}
        runs = {}
        for method in (("mis", "erk") if prec == P.rtbte.FP64 else ("mis",)):
            y = y0.clone()
            t = torch.zeros(1, dtype=torch.float64, device=dev)
            h = torch.zeros(1, dtype=torch.float64, device=dev)
            ctx.reset()
            if method == "mis":   # warm-up on a copy (first launches)
                yw, tw, hw_ = y0.clone(), torch.zeros_like(t), torch.zeros_like(h)
                ctx.step_multirate(yw, tw, hw_, hs, hs)
                ctx.reset()
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            if method == "mis":
                ctx.step_multirate(y, t, h, args.si_t_end, hs)
            else:
                ctx.step_adaptive(y, t, h, args.si_t_end)
            torch.cuda.synchronize()
            wall = time.perf_counter() - w0
            st = ctx.stats()
            runs[method] = y.cpu().numpy()
            leg[method] = {"wall_s": wall, "sim_ps_per_s": args.si_t_end * 1e-3 / wall,
                           "rhs_eph": st["n_rhs_eph"], "rhs_phph": st["n_rhs_phph"],
                           "steps": st["n_accept"], "rejected": st["n_reject"]}
            log(f"[bench] si3d {name} {method}: {args.si_t_end:g} fs in {wall * 1e3:.1f} ms "
                f"({st['n_rhs_eph']} fast-part and {st['n_rhs_phph']} ph-ph evaluations)")
        if "erk" in runs:
            leg["speedup_mis_vs_erk"] = leg["erk"]["wall_s"] / leg["mis"]["wall_s"]
            leg["max_abs_diff_mis_vs_erk"] = float(np.max(np.abs(runs["mis"] - runs["erk"])))
            res["_mis_fp64_y"] = runs["mis"]
        else:
            leg["max_abs_diff_vs_fp64_mis"] = float(np.max(np.abs(runs["mis"] - res["_mis_fp64_y"])))
            leg["speedup_vs_fp64_mis"] = res["fp64"]["mis"]["wall_s"] / leg["mis"]["wall_s"]
        res[name] = leg
        del ctx
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    res.pop("_mis_fp64_y")
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = si3d_cpu_baseline(np, wl, args.si_sample_rows)
    return res


def si3d_cpu_baseline(np, wl, n_rows, seed=5):
    """The FP64 oracle on a sample of the silicon-like workload's rows: the
    entries that feed `n_rows` rows drawn at random (electron and phonon rows
    in proportion), one right-hand side of that sub-problem (median of three),
    as channels per second over the channels it sums."""
    from __graft_entry__ import _ensure_built
    _ensure_built(need_oracle=True)
    import oracle
    prob = wl.problem_arrays()
    rng = np.random.default_rng(seed)
    rows = rng.choice(wl.n_y, size=min(n_rows, wl.n_y), replace=False)
    re_ = rows[rows < wl.n_el]
    rp = rows[rows >= wl.n_el] - wl.n_el
    me = np.zeros(wl.n_el, bool)
    me[re_] = True
    mp = np.zeros(wl.n_ph, bool)
    mp[rp] = True
    ke = me[prob["eph_row"]] | mp[prob["eph_phonon"]]
    kp = mp[prob["pp_row"]]
    sub = dict(prob)
    for k in ("eph_row", "eph_partner", "eph_phonon", "eph_g2"):
        sub[k] = np.ascontiguousarray(prob[k][ke])
    for k in ("pp_row", "pp_a", "pp_b", "pp_v2"):
        sub[k] = np.ascontiguousarray(prob[k][kp])
    o = oracle.Oracle(sub)
    ch = sum(o.counts())
    o.rhs(wl.y0)                                  # first touch of the lists
    reps = 0
    t0 = time.perf_counter()
    while reps < 3 or time.perf_counter() - t0 < 3.0:
        o.rhs(wl.y0)
        reps += 1
    el = (time.perf_counter() - t0) / reps
    return {"value": ch / el, "unit": "channels/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(rows)} random rows of {wl.n_y} ({len(re_)} electron, {len(rp)} phonon): the "
                      f"{ch} channels that feed them, {reps} right-hand sides of {el:.3f} s each"}


def batched_leg(P, torch, np, args):
    """Many independent graphene-like instances (grid sides uniform in
    24..72, initial electron temperatures uniform in 500..3000 K, phonons at
    300 K), each with its own adaptive step (rtol as above), advanced from
    their initial states to the same end time: all in one mixed-precision
    context (launch shape chosen by the autotuner at create, step sequence
    replayed through HIP graphs), against the same instances run one by one
    in plain FP64 contexts.  Simulated time is counted per instance
    (instance-ps per wall second).  Accuracy, untimed: both end states
    against an FP64 batch run at the reference tolerance, per instance; and
    the precision error alone, batched mixed against batched FP64 on the same
    fixed RK4 steps to 1 ps, per instance."""
    import synth
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    ws = synth.build_batch(args.batch, (24, 72), (500.0, 3000.0))
    gen_s = time.perf_counter() - t0
    n = len(ws)
    y0 = np.concatenate([w.y0 for w in ws])
    y0_d = torch.tensor(y0, dtype=torch.float64, device=dev)
    probs = [w.problem_arrays() for w in ws]
    tol = dict(rtol=args.rtol, atol_el=1e-9, atol_ph=1e-12)
    t0 = time.perf_counter()
    ctx = P.Context(probs, precision=P.rtbte.MIXED, use_graph=1, tune=0 if args.no_tune else 1,
                    tiled=args.tiled, **tol)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    counts = ctx.counts()
    C = sum(counts)
    CS = sum(ctx.stored_counts())
    src, tuned_ms = ctx.tuning_source()
    shape = ctx.tuning()
    log(f"[bench] batched: {n} instances, {C} channels ({counts}; {CS} stored), generated {gen_s:.1f} s, "
        f"created {create_s:.1f} s, shape {shape} (source {src}, {tuned_ms:.3f} ms per RHS)")
    y = y0_d.clone()
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    ctx.step_adaptive(y, t, h, 2.0)          # warm-up (first launches, graph capture)
    torch.cuda.synchronize()
    y.copy_(y0_d)
    t.zero_()
    h.zero_()
    ctx.reset()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ctx.step_adaptive(y, t, h, args.batch_t_end)
    torch.cuda.synchronize()
    wall_m = time.perf_counter() - w0
    steps_m = sum(ctx.stats(i)["n_accept"] + ctx.stats(i)["n_reject"] for i in range(n))
    ym = y.cpu().numpy()
    # the batched collision kernel alone, HIP-event timed (after two
    # untimed launches)
    out = torch.empty_like(y)
    for _ in range(2):
        ctx.rhs(y, out, P.PART_ALL)
    ctx.profile(True)
    for _ in range(20):
        ctx.rhs(y, out, P.PART_ALL)
    k_ms, k_n, k_bytes = ctx.profile_read()
    ctx.profile(False)
    kms = k_ms / max(k_n, 1)
    achieved = k_bytes / max(k_n, 1) / (kms * 1e-3) / 1e9
    layouts = [ctx.layout(i) for i in range(n)]
    # precision alone: fixed RK4 steps, the same in both precisions
    n_rk4 = int(round(args.batch_rk4_fs / args.batch_rk4_h))
    y.copy_(y0_d)
    t.zero_()
    ctx.step_rk4(y, t, args.batch_rk4_h, n_rk4)
    torch.cuda.synchronize()
    ym_rk4 = y.cpu().numpy()
    del ctx, y, out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"[bench] batched mixed: {n} x {args.batch_t_end:g} fs in {wall_m * 1e3:.1f} ms ({steps_m} attempts)")
    # FP64 batch: the reference run (tight tolerance) and the same RK4 steps
    ref_tol = dict(rtol=args.ref_rtol, atol_el=1e-12, atol_ph=1e-15)
    c64 = P.Context(probs, use_graph=1, **ref_tol)
    y = y0_d.clone()
    t = torch.zeros(n, dtype=torch.float64, device=dev)
    h = torch.zeros(n, dtype=torch.float64, device=dev)
    c64.step_adaptive(y, t, h, args.batch_t_end)
    torch.cuda.synchronize()
    yref = y.cpu().numpy()
    y.copy_(y0_d)
    t.zero_()
    c64.step_rk4(y, t, args.batch_rk4_h, n_rk4)
    torch.cuda.synchronize()
    y64_rk4 = y.cpu().numpy()
    del c64, y
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # plain FP64, one instance at a time
    wall_f = 0.0
    steps_f = 0
    err_m, err_f, err_rk4 = [], [], []
    for i, w in enumerate(ws):
        c = P.Context(w.problem_arrays(), **tol)
        yi = torch.tensor(w.y0, dtype=torch.float64, device=dev)
        ti = torch.zeros(1, dtype=torch.float64, device=dev)
        hi = torch.zeros(1, dtype=torch.float64, device=dev)
        if i == 0:                                  # warm-up once (first launches)
            c.step_adaptive(yi, ti, hi, 2.0)
            torch.cuda.synchronize()
            yi.copy_(torch.tensor(w.y0, dtype=torch.float64, device=dev))
            ti.zero_()
            hi.zero_()
            c.reset()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        c.step_adaptive(yi, ti, hi, args.batch_t_end)
        torch.cuda.synchronize()
        wall_f += time.perf_counter() - w0
        st = c.stats()
        steps_f += st["n_accept"] + st["n_reject"]
        off, ne, nph = layouts[i]
        sl = slice(off, off + ne + nph)
        err_m.append(float(np.max(np.abs(ym[sl] - yref[sl]))))
        err_f.append(float(np.max(np.abs(yi.cpu().numpy() - yref[sl]))))
        err_rk4.append(float(np.max(np.abs(ym_rk4[sl] - y64_rk4[sl]))))
        del c
    # maxima that a non-finite entry makes non-finite (Python's max skips NaN)
    mx_m, mx_f, mx_rk4 = (float(np.max(np.asarray(e))) for e in (err_m, err_f, err_rk4))
    log(f"[bench] plain FP64: {n} x {args.batch_t_end:g} fs in {wall_f * 1e3:.1f} ms ({steps_f} attempts); "
        f"max |y - y_ref| at {args.batch_t_end:g} fs: batched mixed {mx_m:.2e}, plain FP64 {mx_f:.2e}; "
        f"mixed vs FP64 after {args.batch_rk4_fs:g} fs of RK4: {mx_rk4:.2e}")
    inst_ps = n * args.batch_t_end * 1e-3
    res_cpu = None
    if not args.no_cpu_baseline:
        res_cpu = batched_cpu_baseline(np, ws)
        res_cpu["gpu_batched_kernel_channels_per_s"] = C / (kms * 1e-3)
    return {
        "workload": f"{n} graphene-like instances, sides uniform in 24..72, T_el uniform in 500..3000 K, "
                    f"adaptive Zonneveld ERK rtol {args.rtol:g}, each from its initial state to "
                    f"{args.batch_t_end:g} fs",
        "channels": C, "stored_channels": CS, "channels_eph": counts[0], "channels_phe": counts[1],
        "channels_phph": counts[2],
        "launch_shape": {"rows_per_group_el": shape[0], "rows_per_group_ph": shape[1],
                         "channels_per_item": shape[2],
                         "tuning_source": {0: "default", 1: "tuned at create", 2: "tune cache"}[src],
                         "tuned_rhs_ms": tuned_ms},
        "mixed_graph_wall_s": wall_m, "plain_fp64_wall_s": wall_f,
        "sim_instance_ps_per_s_mixed_batched": inst_ps / wall_m,
        "sim_instance_ps_per_s_plain_fp64": inst_ps / wall_f,
        "speedup_sim_ps_per_s": wall_f / wall_m,
        "attempts_mixed": steps_m, "attempts_plain_fp64": steps_f,
        "reference": dict(ref_tol, note="the batch in FP64, adaptive ERK, to the same end time"),
        "max_abs_err_vs_reference_mixed_batched": mx_m,
        "max_abs_err_vs_reference_plain_fp64": mx_f,
        "err_vs_reference_per_instance_mixed_batched": err_m,
        "err_vs_reference_per_instance_plain_fp64": err_f,
        "precision_check": {"what": f"batched mixed vs batched FP64, the same fixed RK4 steps of "
                                    f"{args.batch_rk4_h:g} fs to {args.batch_rk4_fs:g} fs: max |dy| per instance",
                            "max_abs": mx_rk4, "bar": 1e-6, "per_instance": err_rk4,
                            "all_within_bar": bool(np.all(np.isfinite(err_rk4)) and mx_rk4 <= 1e-6)},
        "roofline_batched_mixed_kernel": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                                          "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                                          "avg_launch_ms": kms, "algorithmic_bytes_per_launch": k_bytes / max(k_n, 1)},
        "generate_s": gen_s, "create_s": create_s,
        "cpu_baseline": res_cpu,
    }


def batched_cpu_baseline(np, ws, every=8, reps=3):
    """The FP64 oracle's right-hand side on a sample of the batch (every
    `every`-th instance, each at its initial state, `reps` evaluations after
    its lists are built), in summed channels per second."""
    from __graft_entry__ import _ensure_built
    _ensure_built(need_oracle=True)
    import oracle
    sample = ws[::every]
    ch, el = 0, 0.0
    for w in sample:
        o = oracle.Oracle(w.problem_arrays())
        t0 = time.perf_counter()
        for _ in range(reps):
            r = o.rhs(w.y0)
        el += time.perf_counter() - t0
        assert np.all(np.isfinite(r))
        ch += reps * sum(o.counts())
        del o
    return {"value": ch / el, "unit": "channels/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"{len(sample)} of the {len(ws)} instances (every {every}th; sides "
                      f"{', '.join(str(w.grid['L']) for w in sample)}), {reps} right-hand sides each at the "
                      f"initial state ({el:.2f} s; list builds untimed); summed channels"}


def timed_steps(ctx, wl, args, C, label, start=None):
    """Warm-up steps from the initial state, then exactly `steps` accepted
    adaptive ERK steps, with the collision kernel timed by HIP events on its
    stream.  With `start` (another leg's state after its warm-up: y, t, h and
    the controller state), the timed steps resume from that state instead, so
    two legs advance from the same point with the same step-size history."""
    import torch
    dev = torch.device("cuda:0")
    y = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    h = torch.zeros(1, dtype=torch.float64, device=dev)   # starting-step estimate
    for i in range(args.warmup):
        ctx.step_adaptive(y, t, h, 1e12, one_step=True)
    torch.cuda.synchronize()
    log(f"[bench] {label} warmup done: t = {t.item():.4g} fs, h = {h.item():.4g} fs")
    if start is None:
        snap = (y.clone(), t.clone(), h.clone(), ctx.get_state())
    else:
        y.copy_(start[0]); t.copy_(start[1]); h.copy_(start[2])
        ctx.set_state(start[3])
        torch.cuda.synchronize()
        snap = start
        log(f"[bench] {label} resumes the first leg's state: t = {t.item():.4g} fs, h = {h.item():.4g} fs")
    s0 = ctx.stats()
    t_start = t.item()
    ctx.profile(True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(args.steps):
        ctx.step_adaptive(y, t, h, 1e12, one_step=True)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    k_ms, k_n, k_bytes = ctx.profile_read()
    ctx.profile(False)
    s1 = ctx.stats()
    t_end = t.item()
    wall = w1 - w0
    evals = s1["n_rhs_eph"] - s0["n_rhs_eph"]
    attempts = (s1["n_accept"] + s1["n_reject"]) - (s0["n_accept"] + s0["n_reject"])
    log(f"[bench] {label}: {args.steps} steps ({attempts} attempts, {evals} RHS) in {wall * 1e3:.1f} ms; "
        f"t {t_start:.4g} -> {t_end:.4g} fs")
    avg_ms = k_ms / max(k_n, 1)
    per_launch = k_bytes / max(k_n, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    kernel = {
        "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "kernel": ("k_items_mixed" if label == "mixed" else "k_items") + " (collision integrals: per-item row sums)",
        "launches": k_n, "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": per_launch,
    }
    return dict(value=evals * C / wall, ms_per_step=wall * 1e3 / args.steps, rhs_per_step=evals / args.steps,
                sim_ps_per_s=(t_end - t_start) * 1e-3 / wall, kernel=kernel, y=y, start=snap,
                t_span=(t_start, t_end))


def mixed_errors(P, torch, np, ctx64, ctx_m, wl, o, args):
    """Accuracy of the mixed path (untimed): the right-hand-side error after
    each of the first steps of a mixed adaptive run (against the oracle, or the
    FP64 GPU path when the oracle is not built), and the largest population
    difference after 1 ps of RK4 with the same 4 fs steps in both precisions."""
    dev = torch.device("cuda:0")
    y = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    h = torch.zeros(1, dtype=torch.float64, device=dev)
    out = torch.empty_like(y)
    ref_d = torch.empty_like(y)
    errs = []
    for i in range(args.err_steps):
        ctx_m.step_adaptive(y, t, h, 1e12, one_step=True)
        ctx_m.rhs(y, out, P.PART_ALL)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
        if o is not None:
            ref = o.rhs(y.cpu().numpy())
        else:
            ctx64.rhs(y, ref_d, P.PART_ALL)
            torch.cuda.synchronize()
            ref = ref_d.cpu().numpy()
        errs.append({"t_fs": t.item(), "normwise": float(np.linalg.norm(g - ref) / np.linalg.norm(ref))})
    log(f"[bench] mixed RHS error per step: {[round(e['normwise'], 9) for e in errs]}")
    res = {}
    for name, c in (("fp64", ctx64), ("mixed", ctx_m)):
        yy = torch.tensor(wl.y0, dtype=torch.float64, device=dev)
        tt = torch.zeros(1, dtype=torch.float64, device=dev)
        c.step_rk4(yy, tt, 4.0, 250)
        torch.cuda.synchronize()
        res[name] = yy.cpu().numpy()
    d = float(np.max(np.abs(res["mixed"] - res["fp64"])))
    log(f"[bench] mixed vs FP64 populations after 1 ps of RK4 (4 fs): {d:.3e}")
    return {"rhs_err_per_step": errs, "rhs_err_reference": "oracle" if o is not None else "FP64 GPU path",
            "pop_err_after_1ps_rk4_4fs": d}


if __name__ == "__main__":
    main()
