"""Throughput of the incompressible Navier-Stokes step on one MI355X.

Workload: the 512^3 lid-driven cavity (Re 1000, dt 3e-4, gamma 0.5,
omega 1.7, tol 1e-8, 200 red-black SOR sweeps per step), state resident in
HBM, synthetic start (fluid at rest, lid (1,0,0) on z = 1).  Each timed
step is the whole step (boundary fill, predictor, rhs, Poisson solve,
projection).  ``value`` is the FP32-mixed form (FP32 fields and sweeps,
FP64 pressure, norms and defect correction); the FP64 form is measured on
the same grid and reported beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 512] [--no-cpu]

Prints one JSON line.  ``roofline`` covers the dominant kernel (the fused
red-black sweep): algorithmic bytes per launch over its average duration,
measured with HIP events on the handle's stream inside the timed region.
``cpu_baseline`` times the FP64 oracle on two full steps of the same
workload on this host; the GPU's FP64 and mixed forms run the same two
steps and their errors against the oracle are reported
(``errors_vs_oracle``), as is the mixed form's error against the FP64 form
over the warmup and timed steps (``mixed_vs_fp64``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1201_2118_amd", "csrc")
# sources that define the sweep kernels (a traffic figure is only reported
# for the exact kernel its counters were taken on)
SWEEP_SOURCES = ("sor_pass.hip", "pass_tile.h", "sor_fused.hip", "ns_internal.h", "reduce.h")
METRIC = "Mcell-steps/s and HBM GB/s, 512^3 NS step, FP32-mixed vs FP64 on 1 GPU"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measure(prm, steps, warmup, keep_state=False):
    """Throughput of K steps on a handle without stage timers (HIP events
    around every launch would add their own gaps to the step), then the
    per-stage and per-launch figures from a second handle of the same grid
    with NS_TIMING (same sweep shape: the autotuner caches it per grid).
    keep_state: also return the final u, v, w of the timed handle (FP64
    device tensors) for the error legs."""
    import torch

    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver

    s = Solver(dict(prm, flags=0), device="cuda:0")
    if warmup:
        s.step(warmup)
    torch.cuda.synchronize()
    a = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    b = time.perf_counter()
    st = s.stats()
    final = [s.get(f) for f in "uvw"] if keep_state else None
    s.close()
    del s
    torch.cuda.empty_cache()

    tsteps = min(steps, 2)
    s = Solver(dict(prm, flags=abi.NS_TIMING), device="cuda:0")
    s.step(1)
    t0 = s.timing()
    s.step(tsteps)
    t1 = s.timing()
    tile = [t1.sor_tile[0], t1.sor_tile[1]]
    s.close()
    n = prm["nx"] * prm["ny"] * prm["nz"]
    secs = b - a
    sor_ms = t1.ms[abi.NS_T_SOR] - t0.ms[abi.NS_T_SOR]
    sor_launches = t1.launches[abi.NS_T_SOR] - t0.launches[abi.NS_T_SOR]
    sor_bytes = t1.sor_bytes - t0.sor_bytes
    stage_ms = {name: (t1.ms[i] - t0.ms[i]) / tsteps for name, i in
                (("bc", abi.NS_T_BC), ("fgh", abi.NS_T_FGH), ("rhs", abi.NS_T_RHS),
                 ("sor", abi.NS_T_SOR), ("defect", abi.NS_T_DEFECT), ("project", abi.NS_T_PROJECT),
                 ("other", abi.NS_T_OTHER))}
    return {
        "mcells": n * steps / secs / 1e6,
        "ms_per_step": secs * 1e3 / steps,
        "sor_avg_ms": sor_ms / max(sor_launches, 1),
        "sor_launches_per_step": sor_launches / tsteps,
        "sor_gbs": sor_bytes / (sor_ms * 1e-3) / 1e9 if sor_ms > 0 else 0.0,
        "sor_bytes_per_launch": sor_bytes / max(sor_launches, 1),
        "stage_ms": stage_ms,
        "stats": st,
        "tile": tile,
        "final": final,
    }


def copy_bandwidth(gib=2.0, reps=5):
    """Device-to-device copy rate (read + write bytes / time) of a plain
    torch copy on this GPU: the practical HBM ceiling the sweep is set
    against, beside the 8 TB/s specification."""
    import torch

    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    secs = e0.elapsed_time(e1) * 1e-3
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 * reps / secs / 1e9


def measure_batched(steps):
    """The batched workload: 64 cavities (sizes U{24..96}, Re U[50, 1000],
    seed 4), adaptive dt (tau 0.5), FP32-mixed, one handle: every step of
    every cavity in one persistent launch.  Throughput on a handle without
    timers; the sweep figures from one timed step of a second persistent
    handle (the slowest team's time in Poisson solves, and the algorithmic
    sweep bytes of all cavities: 12 B per cell per sweep); the multi-launch
    form (one launch per stage and per pass, host-polled) timed beside it."""
    import torch

    import nsworkloads as W
    from paper_1201_2118_amd import abi
    from paper_1201_2118_amd.solver import Solver

    prms, _ = W.batched_64()
    cells = sum(p["nx"] * p["ny"] * p["nz"] for p in prms)

    def run(flags, nsteps):
        s = Solver([dict(p, precision="mixed", flags=flags) for p in prms], device="cuda:0")
        s.step(1)
        torch.cuda.synchronize()
        a = time.perf_counter()
        s.step(nsteps)
        torch.cuda.synchronize()
        b = time.perf_counter()
        sweeps = sum(s.stats(i)["sweeps_total"] for i in range(len(prms)))
        steps_done = sum(s.stats(i)["steps"] for i in range(len(prms)))
        s.close()
        del s
        torch.cuda.empty_cache()
        return b - a, sweeps / steps_done

    secs, mean_sweeps = run(0, steps)
    s = Solver([dict(p, precision="mixed", flags=abi.NS_TIMING if i == 0 else 0) for i, p in enumerate(prms)],
               device="cuda:0")
    s.step(1)
    t0 = s.timing()
    s.step(1)
    t1 = s.timing()
    s.close()
    sor_ms = t1.ms[abi.NS_T_SOR] - t0.ms[abi.NS_T_SOR]
    sor_bytes = t1.sor_bytes - t0.sor_bytes
    all_ms = sum(t1.ms[k] - t0.ms[k] for k in range(abi.NS_T_COUNT))
    ml_secs, _ = run(abi.NS_BATCH_LAUNCHES, max(2, steps // 2))
    sweep_gbs = sor_bytes / (sor_ms * 1e-3) / 1e9 if sor_ms > 0 else None
    return {"value": round(cells * steps / secs / 1e6, 2), "unit": "Mcell-steps/s", "instances": len(prms),
            "cells": cells, "steps": steps, "ms_per_step": round(secs * 1e3 / steps, 3),
            "launch": "persistent (one cooperative launch per ns_step call)",
            "mean_sweeps_per_instance_step": round(mean_sweeps, 1),
            "sweep_ms_per_step": round(sor_ms, 3), "step_ms_timed": round(all_ms, 3),
            "sor_gbs": round(sweep_gbs, 1) if sweep_gbs else None,
            "sor_frac": round(sweep_gbs / PEAK_HBM_GBS, 4) if sweep_gbs else None,
            "multi_launch_value": round(cells * max(2, steps // 2) / ml_secs / 1e6, 2),
            "precision": "mixed", "dt": "adaptive (tau 0.5)"}


def sweep_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel_tag, tile):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE runs, calibrated by a plain copy),
    or None when the summary was taken on other kernel sources or shape."""
    path = os.path.join(PROFILES, f"{kernel_tag}_cavity512_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != sweep_source_hash():
        return None
    if [int(x) for x in kv.get("tile", "0 0").split()] != list(tile):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def step_bytes(n, sweeps, mixed, outers=1, per_launch=1):
    """Algorithmic HBM bytes of one step (minimum single pass per launch):
    FP64 112 + 24 L, mixed 60 + 12 L + 28 O per cell, with L = S / k sweep
    launches for S sweeps done k per launch (k = 1 gives the one-sweep model
    of 112 + 24 S and 60 + 12 S + 28 O)."""
    launches = -(-sweeps // per_launch)
    if mixed:
        return n * (60 + 12 * launches + 28 * outers)
    return n * (112 + 24 * launches)


def unknowns(prm, comp):
    """Slices (k, j, i) of the unknowns of velocity component comp (0, 1, 2)
    or of the cells (3) in the padded layout: faces 1..n-1 along a wall axis
    normal to the component, 1..n otherwise."""
    n = [prm["nx"], prm["ny"], prm["nz"]]
    bc = prm.get("bc", (0, 0, 0))
    hi = list(n)
    if comp < 3 and not bc[comp]:
        hi[comp] -= 1
    return (slice(1, hi[2] + 1), slice(1, hi[1] + 1), slice(1, hi[0] + 1))


def velocity_error(a, b, prm):
    """max over the components of max |a - b| over that component's unknowns,
    divided by the velocity scale of b (max |b| over all three); a, b are
    sequences (u, v, w) of torch tensors or numpy arrays.  Also returns the
    same per component relative to the component's own max |b|."""
    scale, diff, own = 0.0, [], []
    for c in range(3):
        sl = unknowns(prm, c)
        x, y = a[c][sl], b[c][sl]
        d = float(abs(x - y).max())
        m = float(abs(y).max())
        scale = max(scale, m)
        diff.append(d)
        own.append(d / m if m > 0 else d)
    return max(diff) / (scale if scale > 0 else 1.0), own


def pressure_error(a, b, prm):
    sl = unknowns(prm, 3)
    x = a[sl] - a[sl].mean()
    y = b[sl] - b[sl].mean()
    return float(abs(x - y).max() / abs(y).max())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_leg(prm, nsteps=2):
    """The FP64 oracle, untuned, on this host: ``nsteps`` full steps of the
    workload from rest (every sweep of every step), timed as the CPU
    baseline; the GPU's FP64 and mixed forms run the same steps from the
    same start and are compared with it (velocity relative to the velocity
    scale, pressure after mean removal)."""
    import torch

    import oracle
    from paper_1201_2118_amd.solver import Solver

    o = oracle.Oracle(dict(prm, precision="fp64"))
    a = time.perf_counter()
    rc = o.run(nsteps)
    secs = time.perf_counter() - a
    if rc != 0:
        raise RuntimeError(f"oracle run failed ({rc})")
    ref = [o.field(f) for f in "uvw"]
    n = prm["nx"] * prm["ny"] * prm["nz"]
    errs = {"steps": nsteps, "oracle_sweeps": int(o.stats.sweeps_total)}
    for form in ("fp64", "mixed"):
        s = Solver(dict(prm, precision=form, flags=0), device="cuda:0")
        s.step(nsteps)
        got = [s.get_np(f) for f in "uvw"]
        vel, own = velocity_error(got, ref, prm)
        errs[form] = {"vel_rel": vel, "vel_rel_own_max": own,
                      "p_rel": pressure_error(s.get_np("p"), o.p, prm),
                      "sweeps": int(s.stats()["sweeps_total"])}
        s.close()
        del s, got
        torch.cuda.empty_cache()
    base = {"value": n * nsteps / secs / 1e6, "unit": "Mcell-steps/s", "cores": oracle.threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"{nsteps} full steps of the {prm['nx']}^3 workload from rest "
                      f"({int(o.stats.sweeps_total)} sweeps, {secs:.1f} s), FP64; the run the "
                      f"errors_vs_oracle figures compare against"}
    del o
    return base, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["mixed", "fp64", "both"], default="both")
    ap.add_argument("--tile", type=int, nargs=2, default=None,
                    help="fixed sweep shape (rows, z chunk) instead of the autotuned one")
    ap.add_argument("--batched-steps", type=int, default=10,
                    help="steps of the 64-cavity batched workload to time (0 = skip)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="after the runs, copy this many GiB device-to-device once (a plain copy of "
                         "known size that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the one-GPU share of an 8-way z-slab split (512 x 512 x 64, mixed)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched workload (--batched-steps steps) and print its figures "
                         "as one JSON line (for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the domain would be "
              "split into z slabs with halo exchange). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.batched_only:
        print(json.dumps(measure_batched(max(args.batched_steps, 1))), flush=True)
        return

    import nsworkloads as W

    prm, _ = W.cavity_512()
    if args.n != 512:
        prm = W.cavity(args.n, re=1000.0, dt=3e-4, tol=1e-8)
    n = prm["nx"] * prm["ny"] * prm["nz"]
    res = {}
    for form in (["mixed", "fp64"] if args.only == "both" else [args.only]):
        log(f"{form}: {args.n}^3, warmup {args.warmup}, steps {args.steps}")
        cfg = dict(prm, precision=form)
        if args.tile:
            # FP64 two-sweep tiles have 16 rows
            rows = args.tile[0] if form == "mixed" or args.tile[0] <= 16 else 16
            cfg["tile"] = (rows, args.tile[1])
        r = measure(cfg, args.steps, args.warmup, keep_state=args.only == "both")
        st = r["stats"]
        sweeps = st["sweeps_total"] / max(st["steps"], 1)
        k = 2 if r["tile"][0] >= 16 else 1
        o = max(st["outer_max"], 1)
        r["alg_gbs"] = step_bytes(n, sweeps, form == "mixed", o, k) / (r["ms_per_step"] * 1e-3) / 1e9
        r["one_sweep_gbs"] = step_bytes(n, sweeps, form == "mixed", o, 1) / (r["ms_per_step"] * 1e-3) / 1e9
        log(f"{form}: {r['mcells']:.1f} Mcell-steps/s, {r['ms_per_step']:.1f} ms/step, "
            f"sor {r['sor_avg_ms']:.3f} ms/launch = {r['sor_gbs']:.0f} GB/s")
        res[form] = r
    head = res.get("mixed") or res["fp64"]
    dom = head
    f32 = head is res.get("mixed")
    per_launch = 2 if dom["tile"][0] >= 16 else 1
    tag = ("sor_pass" if per_launch == 2 else "sor_fused") + ("_f32" if f32 else "_f64")
    traffic = traffic_from_profile(tag, dom["tile"]) if args.n == 512 else None
    # Algorithmic bytes per launch: 12 (FP32) / 24 (FP64) bytes per cell per
    # sweep times the sweeps one launch does (a two-sweep pass is priced as
    # two sweeps); the bytes of a single pass over the data and the counter
    # traffic are kept beside it.
    one_pass = dom["sor_gbs"]
    achieved = per_launch * one_pass
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": round(traffic) if traffic else None,
            "kernel": "red-black SOR, %d sweep(s) per launch (%s)" % (per_launch, "FP32" if f32 else "FP64"),
            "sweeps_per_launch": per_launch,
            "bytes_per_launch": per_launch * dom["sor_bytes_per_launch"],
            "avg_launch_ms": round(dom["sor_avg_ms"], 5),
            "one_pass_gbs": round(one_pass, 1),
            "one_pass_frac": round(one_pass / PEAK_HBM_GBS, 4),
            "traffic_gbs": round(traffic / (dom["sor_avg_ms"] * 1e-3) / 1e9, 1) if traffic else None,
            "limiter": ("instruction issue and waits: VALU 64% busy, 45% of the wave cycles waiting on "
                        "memory / LDS / the per-plane barrier (SQ counters)") if per_launch == 2 and f32
                       else ("vector-ALU issue (two sweeps per launch)" if per_launch == 2 else "HBM"),
            "tile": dom["tile"]}
    roof["copy_gbs_measured"] = round(copy_bandwidth(), 1)
    out = {
        "metric": METRIC,
        "value": round(head["mcells"], 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head is res.get("mixed") else "f64",
        "data": "synthetic",
        "config": {"workload": f"lid-driven cavity {args.n}^3", "re": prm["re"], "dt": prm["dt"],
                   "gamma": prm["gamma"], "omega": prm["omega"], "tol": prm["tol"],
                   "itermax": prm["itermax"], "precision": "mixed" if head is res.get("mixed") else "fp64"},
        "hbm_gbs_algorithmic": round(head["alg_gbs"], 1),
        "gbs_one_sweep_model": round(head["one_sweep_gbs"], 1),
        "sweeps_per_step": head["stats"]["sweeps_total"] / max(head["stats"]["steps"], 1),
        "stage_ms": {k: round(v, 4) for k, v in head["stage_ms"].items()},
        "roofline": roof,
    }
    if "fp64" in res and head is not res["fp64"]:
        f = res["fp64"]
        out["fp64"] = {"value": round(f["mcells"], 2), "ms_per_step": round(f["ms_per_step"], 3),
                       "hbm_gbs_algorithmic": round(f["alg_gbs"], 1),
                       "gbs_one_sweep_model": round(f["one_sweep_gbs"], 1), "sor_gbs": round(f["sor_gbs"], 1),
                       "sor_avg_ms": round(f["sor_avg_ms"], 5), "tile": f["tile"],
                       "stage_ms": {k: round(v, 4) for k, v in f["stage_ms"].items()}}
    if "fp64" in res and "mixed" in res:
        vel, own = velocity_error(res["mixed"]["final"], res["fp64"]["final"], prm)
        out["mixed_vs_fp64"] = {"steps": args.warmup + args.steps, "vel_rel": vel, "vel_rel_own_max": own,
                                "note": "both forms from rest over the warmup and timed steps; velocity "
                                        "error relative to the FP64 run's velocity scale (and per component "
                                        "relative to its own max)"}
        log(f"mixed vs fp64 after {args.warmup + args.steps} steps: {vel:.2e}")
    for r in res.values():
        r["final"] = None
    import torch
    torch.cuda.empty_cache()
    if not args.no_slab and args.n % 8 == 0:
        # one GPU's share if the cavity were split into 8 z slabs: the same
        # kernels on n x n x n/8 cells (walls at the slab ends stand in for
        # the ghost planes a neighbour would send)
        sl = dict(prm, nz=args.n // 8, lz=prm["lz"] / 8, precision="mixed")
        r = measure(sl, args.steps, args.warmup)
        out["slab_share"] = {"grid": [args.n, args.n, args.n // 8], "precision": "mixed",
                             "value": round(r["mcells"], 2), "unit": "Mcell-steps/s",
                             "ms_per_step": round(r["ms_per_step"], 3), "sor_avg_ms": round(r["sor_avg_ms"], 5),
                             "sor_launches_per_step": r["sor_launches_per_step"], "tile": r["tile"],
                             "stage_ms": {k: round(v, 4) for k, v in r["stage_ms"].items()}}
        log(f"slab share {args.n}x{args.n}x{args.n // 8}: {r['mcells']:.1f} Mcell-steps/s, "
            f"sor {r['sor_avg_ms'] * 1e3:.1f} us/launch")
        torch.cuda.empty_cache()
    if args.batched_steps > 0:
        out["batched"] = measure_batched(args.batched_steps)
        log(f"batched: {out['batched']['value']} Mcell-steps/s over {out['batched']['instances']} cavities")
    if args.copy_probe > 0:
        import torch
        nbytes = int(args.copy_probe * (1 << 30))
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0")
        c = torch.empty_like(a)
        torch.cuda.synchronize()
        c.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nbytes} bytes read, {nbytes} bytes written")
        out["copy_probe_bytes"] = nbytes
        del a, c
    if not args.no_cpu:
        log("oracle leg: cpu baseline and GPU errors against the oracle")
        out["cpu_baseline"], out["errors_vs_oracle"] = oracle_leg(prm)
        log(f"errors vs oracle: {out['errors_vs_oracle']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
