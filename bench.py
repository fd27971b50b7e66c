"""Throughput of the PDG transport sweep + relaxation on one MI355X.

One step = one full implicit transport sweep of every velocity and component
(theta-scheme, Sec. 4.1-4.2) + one relaxation (eq. collision_cn), i.e. the
interior step of the collapsed Strang composition (Sec. 5.1).  The timed
region runs pdg_step(K): T(dt/2) C [T(dt) C]^(K-1) T(dt/2), i.e. K+1 sweep
launches and K relax launches, counted as K steps.  Inputs are resident in
HBM before the timed region.

Prints one JSON line (rank 0 of a single process):
  value      = N_DoF * K / wall time      [DoF-updates/s], N_DoF = nv m Nc (d+1)^D
  roofline   = the sweep kernel (the dominant launch) against the 8 TB/s HBM
               peak: algorithmic bytes per launch = read + write of the state,
               2 s N_DoF (s = 8 B for the binary64 state, 6 B for the 48-bit
               state of binary32 + refinement, 4 B for binary32), over its
               HIP-event launch duration
  precisions = the same measurement for binary64, binary32 + binary64
               refinement on the 48-bit state and on a binary64 state, and
               plain binary32, each with its error against binary64
  cpu_baseline = the CPU oracle timed on a bounded sample of the workload
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "DoF-updates/s per transport+relax step, FP32+refine vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0
PREC_NAMES = {0: "fp64", 3: "fp32refine48", 2: "fp32refine", 1: "fp32"}
# arithmetic of the path: binary32 cell solves + binary64 residual for the refined ones
DTYPE_NAMES = {0: "f64", 3: "f32+f64", 2: "f32+f64", 1: "f32"}
STATE_BYTES = {0: 8, 3: 6, 2: 8, 1: 4}
DEFAULT_WORKLOAD = "euler3d_128"


def inst_dict(inst):
    par = {"advection": lambda p: list(p["a"]), "euler": lambda p: [p["gamma"]],
           "d2q9": lambda p: [p["g"]]}[inst.feq_kind](inst.feq_param)
    return dict(dim=inst.dim, n=list(inst.n), degree=inst.degree, v=np.asarray(inst.vel, float), m=inst.m,
                lo=list(inst.lo), hi=list(inst.hi), feq=inst.feq_kind, feq_param=par,
                edges=getattr(inst, "edges", None))


def initial_state(pdg, prob, insts, torch):
    """f = f^eq(w0) and fb = f^eq(w0 at the inflow points), built on the device.
    w_inflow holds, per instance and velocity, the moments of w0 at the
    velocity's inflow points (m moments, or 3 for the D2Q9 model)."""
    w = np.empty(prob.layout["w_elems"])
    fbw_blocks = []
    for i, inst in enumerate(insts):
        vol, inflow = prob.node_coords(i)
        w[prob.layout["w_off"][i]:prob.layout["w_off"][i + 1]] = inst.w0(vol.reshape(inst.dim, -1).T).ravel()
        ioff = 0
        nc = int(np.prod(inst.n))
        for v in range(inst.vel.shape[0]):
            blocks = []
            for ax in range(inst.dim):
                if inst.vel[v][ax] == 0:
                    continue
                npts = (inst.degree + 1) ** (inst.dim - 1) * (nc // inst.n[ax])
                pts = inflow[ioff:ioff + inst.dim * npts].reshape(inst.dim, npts).T
                blocks.append(inst.w0(pts))
                ioff += inst.dim * npts
            if blocks:
                fbw_blocks.append(np.concatenate(blocks, axis=1).ravel())   # [k][face][t][tau]
    fbw = np.concatenate(fbw_blocks) if fbw_blocks else np.zeros(1)
    f = prob.new_state()   # the prepared precision's storage
    fb = torch.empty(prob.layout["fb_elems"], dtype=torch.float64, device="cuda")
    w_t = torch.from_numpy(w).cuda()
    prob.equilibrium(w_t, f)
    fbw_t = torch.from_numpy(fbw).cuda()
    prob.inflow_equilibrium(fbw_t, fb)
    torch.cuda.synchronize()
    return f, fb, w_t


def kernel_source_hash():
    """Hash of the sources that define the axis-aligned sweep kernel: its
    translation unit, its cell solves, the device helpers, and the part of the
    internal header that holds its item and operator layouts (up to the
    node-local structs)."""
    csrc = os.path.join(ROOT, "paper_1702_00169_amd", "csrc")
    h = hashlib.sha256()
    for name in ("pdg_sweep.hip", "pdg_cellop.h", "pdg_device.h"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(csrc, "pdg_internal.h"), "rb") as fh:
        text = fh.read()
    h.update(text.split(b"// Per-instance data of the node-local kernels.")[0])
    return h.hexdigest()[:16]


def traffic_for(workload, prec_name):
    """HBM bytes per sweep launch from committed rocprofv3 PMC runs, if they
    were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    key = f"{workload}/{prec_name}"
    ent = rec.get(key)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


def record_traffic(workload, prec_name, fetch_csv, write_csv):
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, each with --copy-probe-mib 1024 and fixed --tiles) into HBM
    bytes per sweep launch, and store them in profiles/sweep_traffic.json
    keyed by the sweep kernel's source hash.  Both counters are calibrated on
    the 1 GiB device copy of the same run (it reads and writes 1 GiB)."""
    import csv

    def rows(path):
        with open(path) as fh:
            return list(csv.DictReader(fh))

    f, w = rows(fetch_csv), rows(write_csv)
    copy_bytes = 1024 * 2 ** 20

    def values(rs, name, floor=0.0):
        return [float(r["Counter_Value"]) for r in rs if name in r["Kernel_Name"] and float(r["Counter_Value"]) > floor]

    cf, cw = values(f, "copyBuffer", 1e5), values(w, "copyBuffer", 1e5)
    fetch_factor = copy_bytes / (sum(cf) / len(cf) * 1024)
    write_factor = copy_bytes / (sum(cw) / len(cw) * 1024)
    wl = W.make(workload)
    state_b = {"fp32": 4, "fp32refine48": 6}.get(prec_name, 8)
    alg_write_kib = wl.n_dof * state_b / 1024
    sf, sw = values(f, "sweep_kernel"), values(w, "sweep_kernel")
    # the full sweep launches (steps and timing loop) write the whole state;
    # both runs issue the same dispatch sequence, so they are the same tail
    ntail = 0
    while ntail < len(sw) and abs(sw[-1 - ntail] - alg_write_kib) / alg_write_kib < 0.02:
        ntail += 1
    if ntail == 0:
        raise SystemExit("no full sweep launch found in the counter runs")
    full_f, full_w = sf[len(sf) - ntail:], sw[len(sw) - ntail:]
    fetch_b = sum(full_f) / len(full_f) * 1024 * fetch_factor
    write_b = sum(full_w) / len(full_w) * 1024 * write_factor
    path = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    rec = {}
    if os.path.exists(path):
        with open(path) as fh:
            rec = json.load(fh)
    rec[f"{workload}/{prec_name}"] = {
        "source_hash": kernel_source_hash(), "bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b,
        "write_bytes": write_b, "fetch_factor": fetch_factor, "write_factor": write_factor,
        "full_launches": ntail, "algorithmic_bytes_per_launch": 2 * wl.n_dof * state_b}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec[f"{workload}/{prec_name}"], indent=1))


def measure(pdg, torch, wl, prec, steps, warmup, reps, keep_state=False, autotune=True, tiles=None):
    insts = wl.instances
    prob = pdg.Problem([inst_dict(i) for i in insts])
    prob.prepare(wl.dt, theta=wl.theta, omega=wl.omega, scheme=pdg.PDG_STRANG_COLLAPSED, precision=prec)
    f, fb, w_t = initial_state(pdg, prob, insts, torch)
    if tiles:
        prob.set_tiles(tiles)
    elif autotune:
        # tile search on the state buffer itself, then restore the initial state
        prob.autotune(f, fb, reps=3)
        prob.equilibrium(w_t, f)
        torch.cuda.synchronize()
    del w_t
    tiles = prob.tiles()
    f_init = f.clone() if keep_state else None
    n_dof = wl.n_dof
    # warm-up (also records the step graph)
    if warmup > 0:
        prob.step(f, fb, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.step(f, fb, steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prob.sync_status()   # raises (PDG_EDEVICE) if a dense-path wait gave up: the timed run would be invalid
    refine_corr = prob.last_refine_correction() if prec in (pdg.PDG_FP32_REFINE, pdg.PDG_FP32_REFINE_P48) else None
    # per-launch durations on the stream the kernels run on
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record(stream)
    for _ in range(reps):
        prob.transport_sweep(f, fb, fb, wl.dt)
    ev[1].record(stream)
    for _ in range(reps):
        prob.relax(f)
    ev[2].record(stream)
    torch.cuda.synchronize()
    prob.sync_status()
    t_sweep = ev[0].elapsed_time(ev[1]) / reps * 1e-3
    t_relax = ev[1].elapsed_time(ev[2]) / reps * 1e-3
    state_bytes = STATE_BYTES[prec]
    out = dict(
        value=n_dof * steps / wall, ms_per_step=wall / steps * 1e3, wall_s=wall,
        sweep_us=t_sweep * 1e6, relax_us=t_relax * 1e6,
        sweep_gbs=2 * state_bytes * n_dof / t_sweep / 1e9,
        relax_gbs=2 * state_bytes * n_dof / t_relax / 1e9,
        bytes_per_sweep=2 * state_bytes * n_dof,
        refine_correction=refine_corr,
        tiles=tiles,
    )
    result = None
    if keep_state:
        # the state after warmup + steps from the same initial data, for errors
        g = f_init
        prob.step(g, fb, warmup)
        prob.step(g, fb, steps)
        torch.cuda.synchronize()
        prob.sync_status()
        result = prob.state_to_f64(g)   # binary64 values, on the device
        del g
    del f, fb
    prob.close()
    torch.cuda.empty_cache()
    return out, result


def cpu_baseline(wl_name, seed, target_s):
    """The CPU oracle (as it stands) on a bounded sample of the workload."""
    import threadpoolctl

    from oracle import step as ost
    def one_step(scale):
        wl = W.make(wl_name, seed=seed, scale=scale)
        inst = wl.instances[0]
        edges = None
        if getattr(inst, "edges", None) is not None:
            edges = [np.asarray(e, float) if e is not None else np.linspace(inst.lo[k], inst.hi[k], inst.n[k] + 1)
                     for k, e in enumerate(inst.edges)]
        prob = ost.Problem(inst.n, inst.lo, inst.hi, inst.degree, inst.vel, inst.m, inst.feq_kind, inst.feq_param,
                           edges)
        x = prob.mesh.node_coords().reshape(-1, inst.dim)
        f0 = prob.feq(inst.w0(x).reshape(-1, prob.mesh.nc, prob.mesh.nd))
        fb = prob.inflow_from_w(inst.w0)
        t0 = time.perf_counter()
        f = prob.transport(f0, fb, fb, wl.dt, wl.theta)
        prob.local(f, wl.dt / 2, wl.omega, wl.dt / 2)   # S C S; the source is the identity without one
        return inst, time.perf_counter() - t0

    # calibrate the oracle's rate on a small mesh, then size the sample for ~target_s
    full_n = W.make(wl_name, seed=seed).instances[0].n[0]
    small = min(full_n, 8)
    inst_s, t_s = one_step(small)
    rate = inst_s.n_dof / t_s
    scale = small
    while scale < full_n:
        nxt = min(full_n, scale + max(1, scale // 4))
        if W.make(wl_name, seed=seed, scale=nxt).instances[0].n_dof / rate > target_s:
            break
        scale = nxt
    inst, wall = one_step(scale)
    info = threadpoolctl.threadpool_info()
    threads = max([1] + [int(i.get("num_threads", 1)) for i in info])
    return {"value": inst.n_dof / wall, "unit": "DoF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one interior step (sweep of all {inst.vel.shape[0]} velocities + relax) of {wl_name} "
                      f"shrunk to {'x'.join(map(str, inst.n))} cells ({inst.n_dof} DoF), {wall:.1f} s, "
                      f"numpy/scipy float64; host os.cpu_count()={os.cpu_count()}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=W.WORKLOADS)
    ap.add_argument("--precision", default="fp32refine48", choices=list(PREC_NAMES.values()))
    ap.add_argument("--reps", type=int, default=20, help="launches per kernel-timing loop")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-compare", action="store_true", help="skip the other precisions")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tiles")
    ap.add_argument("--no-fused", action="store_true",
                    help="skip the steps with the opt-in fused collision + x transport (PDG_FUSED=1)")
    ap.add_argument("--tiles", default=None,
                    help="JSON list of tiles ({np, x_kind, C, S}) to apply instead of autotuning (main precision)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="size of the plain device copy (bandwidth reference and counter calibration)")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"), default=None,
                    help="store the HBM traffic of the sweep from two rocprofv3 --pmc runs (no GPU work)")
    args = ap.parse_args()

    if args.record_traffic:
        record_traffic(args.workload, args.precision, *args.record_traffic)
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1702_00169_amd as pdg
    torch.cuda.set_device(0)

    prec_main = {v: k for k, v in PREC_NAMES.items()}[args.precision]
    wl = W.make(args.workload, seed=args.seed)
    compare = not args.no_compare
    precs = [prec_main] + ([p for p in (0, 3, 2, 1) if p != prec_main] if compare else [])
    results, states = {}, {}
    for p in precs:
        print(f"[bench] {args.workload} {PREC_NAMES[p]}: {args.warmup} warm-up + {args.steps} timed steps",
              file=sys.stderr, flush=True)
        results[p], states[p] = measure(pdg, torch, wl, p, args.steps, args.warmup, args.reps, keep_state=compare,
                                        autotune=not args.no_autotune,
                                        tiles=json.loads(args.tiles) if args.tiles and p == prec_main else None)
        print(f"[bench]   {results[p]['value']:.4e} DoF/s, sweep {results[p]['sweep_us']:.1f} us "
              f"({results[p]['sweep_gbs']:.0f} GB/s), relax {results[p]['relax_us']:.1f} us", file=sys.stderr,
              flush=True)
    # the same steps with the opt-in fused collision + x transport (read at
    # prepare), on the tiles chosen above; reported beside the headline
    fused_report = None
    if compare and not args.no_fused:
        fused_report = {}
        old_env = os.environ.get("PDG_FUSED")
        os.environ["PDG_FUSED"] = "1"
        try:
            for p in dict.fromkeys((prec_main, 0)):
                print(f"[bench] {args.workload} {PREC_NAMES[p]} with PDG_FUSED=1: {args.warmup} warm-up + "
                      f"{args.steps} timed steps", file=sys.stderr, flush=True)
                r, _ = measure(pdg, torch, wl, p, args.steps, args.warmup, args.reps, autotune=False,
                               tiles=results[p]["tiles"])
                fused_report[PREC_NAMES[p]] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                               "vs_separate_passes": r["value"] / results[p]["value"]}
                print(f"[bench]   {r['value']:.4e} DoF/s ({r['value'] / results[p]['value']:.3f} x separate passes)",
                      file=sys.stderr, flush=True)
        finally:
            if old_env is None:
                os.environ.pop("PDG_FUSED", None)
            else:
                os.environ["PDG_FUSED"] = old_env
        fused_report["note"] = ("opt-in (PDG_FUSED=1, read at prepare): each collision of the collapsed step runs "
                                "with the x transport in one pass over the state where the instance allows it; "
                                "value above is without it")
    # a plain device copy of the state's size: the practical streaming ceiling
    copy_mib = args.copy_probe_mib or max(256, min(4096, results[prec_main]["bytes_per_sweep"] // 2 // 2 ** 20))
    x = torch.empty(copy_mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * x.numel() * 8 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y

    main_res = results[prec_main]
    prec_report = {}
    ref = states.get(0)
    for p in precs:
        r = dict(results[p])
        entry = {k: r[k] for k in ("value", "ms_per_step", "sweep_us", "relax_us", "sweep_gbs", "relax_gbs")}
        entry["refine_correction"] = r["refine_correction"]
        entry["tiles"] = r["tiles"]
        if ref is not None and p != 0 and states.get(p) is not None:
            # relative errors against the binary64 state, reduced on the device
            d = states[p] - ref
            entry["rel_err_vs_fp64_l2"] = float(torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref))
            entry["rel_err_vs_fp64_max"] = float(d.abs().max() / ref.abs().max())
            del d
        prec_report[PREC_NAMES[p]] = entry
    if ref is not None:
        prec_report["fp64"]["rel_err_note"] = ("fp64 matches the CPU oracle to <= 1e-12 in the parity tests; "
                                               "the other precisions are compared with it after the same steps")
    states.clear()
    ref = None
    torch.cuda.empty_cache()

    traffic = traffic_for(args.workload, PREC_NAMES[prec_main])  # HBM bytes per sweep launch, or None
    # velocities with two or three non-zero components go through the dense tiled sweep
    dense = any(np.count_nonzero(v) >= 2 for inst in wl.instances for v in inst.vel)
    roof = {"bound": "hbm", "achieved": main_res["sweep_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": main_res["sweep_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "transport sweep (sweep_kernel" + (" + dense_sweep_kernel)" if dense else ")"), "algorithmic_bytes_per_launch": main_res["bytes_per_sweep"],
            "launch_us": main_res["sweep_us"], "device_copy_gbs": copy_gbs,
            "traffic_over_algorithmic": (traffic / main_res["bytes_per_sweep"]) if traffic else None,
            "step_bytes_per_dof": 4 * STATE_BYTES[prec_main],
            "step_gbs": main_res["value"] * 4 * STATE_BYTES[prec_main] / 1e9}
    inst0 = wl.instances[0]
    config = {"workload": f"{args.workload}: {wl.description}", "n_dof": wl.n_dof,
              "instances": len(wl.instances), "cells": list(inst0.n) if len(wl.instances) == 1 else "per instance",
              "degree": inst0.degree if len(wl.instances) == 1 else "per instance",
              "nv": int(inst0.vel.shape[0]), "m": inst0.m, "dt": wl.dt, "theta": wl.theta, "omega": wl.omega,
              "scheme": "collapsed Strang" + (" with source" if inst0.feq_kind == "d2q9" else ""),
              "precision": PREC_NAMES[prec_main], "seed": args.seed}
    out = {"metric": METRIC, "value": main_res["value"], "unit": "DoF-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": main_res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": DTYPE_NAMES[prec_main],
           "data": "synthetic", "config": config, "roofline": roof, "precisions": prec_report}
    if fused_report is not None:
        out["fused"] = fused_report
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload if args.workload != "batch96" else "adv2d_16", args.seed,
                                           args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
