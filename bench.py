"""Benchmark of the two-component D3Q19 Shan-Chen evaporation step on one MI355X.

Headline: the 512^3 droplet (radius 120, psi = rho, g = 0.9, tau = 1, sink
rho_H = 0.04 on all six faces) in FP32-shifted storage, MLUPS over the timed
steps (one step = the fused pull/sink/moments/force/collision/store launch;
FP64 diagnostics every --diag-every steps are inside the timed region). It is
the largest configuration that fits one GPU.

Extra forms on the same line:
  - the 128^3 droplet in FP32S, FP64, FP16N, FP16NF and FP16S;
  - the 512^3 droplet in FP64 and in its FP16 variant (FP16N);
  - the 64 batched uneven droplets (48^3..156^3) in one launch per step,
    replayed as HIP graphs, against 64 separate contexts;
  - the films 64x64x512 (FP32S, FP64, FP16N) and 4x4x128 (FP64).
Each reduced-precision form carries its errors against the FP64 GPU run of
the same workload over the same steps; its speed-up over FP64 is reported
only where those errors pass the stated bars (matched accuracy), otherwise
the form is marked as failing them.

Prints one JSON line. Synthetic inputs only (see lbinputs).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2-comp D3Q19 MLUPS + % HBM peak; FP32/FP16/batched vs plain FP64 at stated error"
HBM_PEAK_GBPS = 8000.0
# 2 comps x 19 x (read + write) x element size; FP16N stores the rest
# population in FP32 (2 x 2 x (18 x 2 + 4))
BYTES_PER_LU = {"fp64": 608, "fp32s": 304, "fp16s": 152, "fp16n": 160, "fp16nf": 160}
DTYPE = {"fp64": "f64", "fp32s": "f32", "fp16s": "f32", "fp16n": "f32", "fp16nf": "f32"}
# Accuracy bars against the FP64 run of the same workload and steps: max
# |rho_A - rho_A(FP64)|, and the relative drifts of M^A + M^B and M^A + E.
BARS = {"fp32s": {"max_abs_drho": 1e-5, "mass_drift": 1e-6},
        "fp16n": {"max_abs_drho": 1e-3, "mass_drift": 1e-6},
        "fp16nf": {"max_abs_drho": 1e-3, "mass_drift": 1e-6},
        "fp16s": {"max_abs_drho": 1e-3, "mass_drift": 1e-3}}


def kernel_hash() -> str:
    """Hash of the kernel sources' code (the one the library is built with)."""
    from paper_1701_03637_amd.build import kernel_hash as h
    return h()


def step_kernel_name(tiles, st="StF32S") -> str:
    """Name of the step kernel a resolved schedule (nt, tw, th, nzc, variant)
    launches."""
    nt, variant = tiles[0], tiles[4]
    if variant == 3:
        return f"lbsc::k_step_pipe<lbsc::{st}, {nt}>"
    return f"lbsc::k_step<lbsc::{st}, {nt}, {'false' if variant == 2 else 'true'}>"


def measured_traffic(workload: str, precision: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


_DENSITIES = {}


def densities(w):
    """Initial densities of a workload, computed once per workload."""
    if w.name not in _DENSITIES:
        _DENSITIES.clear()
        _DENSITIES[w.name] = w.densities()
    return _DENSITIES[w.name]


def make_sim(lb, w, precision):
    p = lb.make_params(w.nx, w.ny, w.nz, wall_z=w.wall_z, g=w.g, psi=w.psi, precision=precision, shift=w.shift,
                       sink=w.sink, rho_h=w.rho_h, sink_radius=w.sink_radius, phi_delta=w.phi_delta,
                       flags=lb.FLAG_FP16S_SINK if precision == "fp16s" else 0)
    return lb.Sim(p)


def timed_run(sim, steps, warmup, diag_every, torch):
    """Warm up, then time `steps` steps with HIP events (on the library's
    stream, torch's current stream) around each batch of steps. Returns
    (wall_ms_region, kernel_ms_total, diag)."""
    sim.step(warmup)
    torch.cuda.synchronize()
    step_ms = 0.0
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    done = 0
    diag = None
    while done < steps:
        n = min(diag_every, steps - done) if diag_every > 0 else steps - done
        ev0.record()
        sim.step(n)
        ev1.record()
        done += n
        if diag_every > 0:
            diag = sim.diagnostics()   # synchronises
        else:
            torch.cuda.synchronize()
        step_ms += ev0.elapsed_time(ev1)
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    if diag is None:
        diag = sim.diagnostics()
    return wall_ms, step_ms, diag


def form_single(lb, torch, w, precision, steps, warmup, diag_every, graph, tune_steps, pin=None):
    """Times one workload in one storage form; returns its record and the
    context (the caller closes it)."""
    sim = make_sim(lb, w, precision)
    a, b = densities(w)
    if pin:
        sim.set_tiles(*pin)
    sim.init_from_density(a, b)
    if tune_steps and not pin:
        sim.tune(tune_steps)   # leaves the initial state as it was
    del a, b
    d0 = sim.diagnostics()
    if graph:
        sim.set_graph(graph)
    wall_ms, step_ms, d1 = timed_run(sim, steps, warmup, diag_every, torch)
    lu = w.nodes * steps
    tot0 = d0["mass"][0] + d0["mass"][1]
    out = {
        "workload": w.name, "precision": precision, "nodes": w.nodes, "steps": steps,
        "mlups": lu / (wall_ms * 1e-3) / 1e6,
        "kernel_mlups": lu / (step_ms * 1e-3) / 1e6,
        "ms_per_step": wall_ms / steps,
        "kernel_ms_per_step": step_ms / steps,
        "alg_GBps": w.nodes * BYTES_PER_LU[precision] / (step_ms / steps * 1e-3) / 1e9,
        "mass_drift_rel": abs(d1["mass"][0] + d1["mass"][1] - tot0) / tot0,
        "mass_A_plus_E_drift_rel": abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]) / tot0,
        "r_droplet": d1["r_droplet"],
        "evaporated": d1["evaporated"],
        "items_per_step": sim.num_items(),
        "tiles": list(sim.tiles()),
    }
    out["hbm_frac_alg"] = out["alg_GBps"] / HBM_PEAK_GBPS
    return out, sim


def accuracy_runs(lb, torch, w, forms, steps):
    """Each form and FP64 from the same initial densities over the same
    `steps` steps (graphs of 100 steps): the form's max |drho_A| against
    FP64 and its mass drifts, judged against BARS."""
    a, b = densities(w)

    def run(prec):
        sim = make_sim(lb, w, prec)
        sim.init_from_density(a, b)
        d0 = sim.diagnostics()
        sim.set_graph(100 if steps >= 200 else 0)
        sim.step(steps)
        d1 = sim.diagnostics()
        rho = sim.density(0)
        sim.close()
        tot0 = d0["mass"][0] + d0["mass"][1]
        drift = max(abs(d1["mass"][0] + d1["mass"][1] - tot0), abs(d1["mass"][0] + d1["evaporated"] - d0["mass"][0]))
        return rho, drift / tot0

    ref, drift64 = run("fp64")
    out = {"steps": steps, "fp64_mass_drift": drift64}
    for prec in forms:
        rho, drift = run(prec)
        err = float((rho - ref).abs().max())
        del rho
        ok = err <= BARS[prec]["max_abs_drho"] and drift <= BARS[prec]["mass_drift"]
        out[prec] = {"max_abs_drho_vs_fp64": err, "mass_drift": drift, "bars": BARS[prec], "pass": ok}
    del ref
    torch.cuda.empty_cache()
    return out


def speedup_at_matched_accuracy(rec, fp64_rec, acc):
    """Speed-up over FP64 only where the form passed its accuracy bars."""
    if acc is None or fp64_rec is None:
        return
    a = acc.get(rec["precision"])
    if a is None:
        return
    rec["accuracy"] = a
    if a["pass"]:
        rec["speedup_vs_fp64"] = rec["mlups"] / fp64_rec["mlups"]
    else:
        rec["speedup_vs_fp64"] = None
        rec["accuracy_failed"] = "errors against FP64 exceed the bars; no speed-up is claimed"


def form_batched(lb, torch, steps, warmup, graph, tune_steps):
    import lbinputs as li
    ws = li.batch64()
    params = [lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink, rho_h=w.rho_h)
              for w in ws]
    sim = lb.Sim(params)
    dens = [w.densities() for w in ws]
    for k, (a, b) in enumerate(dens):
        sim.init_from_density(a, b, inst=k)
    if tune_steps:
        sim.tune(tune_steps)
    nodes = sum(w.nodes for w in ws)
    m0 = []
    for k in range(len(ws)):
        d = sim.diagnostics(inst=k)
        m0.append((d["mass"][0], d["mass"][0] + d["mass"][1]))
    if graph:
        sim.set_graph(graph)
    sim.step(warmup)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    sim.step(steps)
    ev1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    step_ms = ev0.elapsed_time(ev1)
    drift = 0.0
    for k in range(len(ws)):
        d = sim.diagnostics(inst=k)
        drift = max(drift, abs(d["mass"][0] + d["mass"][1] - m0[k][1]) / m0[k][1],
                    abs(d["mass"][0] + d["evaporated"] - m0[k][0]) / m0[k][1])
    res = {
        "workload": "batch64 droplets 48^3..156^3 (seed 1)", "precision": "fp32s", "instances": len(ws),
        "nodes": nodes, "steps": steps, "graph_steps": graph,
        "mlups": nodes * steps / (wall_ms * 1e-3) / 1e6,
        "kernel_ms_per_step": step_ms / steps,
        "alg_GBps": nodes * 304 / (step_ms / steps * 1e-3) / 1e9,
        "items_per_step": sim.num_items(),
        "tiles": list(sim.tiles()),
        # per-instance tile width, rows and chunk length picked by the size
        # class tuner (0: the context's), by box side
        "inst_tiles_by_side": {str(w.nx): list(sim.inst_tiles(k))[1:4] for k, w in sorted(
            enumerate(ws), key=lambda kw: kw[1].nx)},
        "max_mass_drift_rel": drift,
    }
    res["hbm_frac_alg"] = res["alg_GBps"] / HBM_PEAK_GBPS
    sim.close()
    # The same 64 boxes as 64 plain contexts stepped one after another (one
    # launch per box and step, default schedules), the alternative batching
    # replaces.
    seq = []
    for w, (a, b) in zip(ws, dens):
        s1 = lb.Sim(lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink,
                                   rho_h=w.rho_h))
        s1.init_from_density(a, b)
        seq.append(s1)
    for s1 in seq:
        s1.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        for s1 in seq:
            s1.step(1)
    ev1.record()
    torch.cuda.synchronize()
    seq_wall_ms = (time.perf_counter() - t0) * 1e3
    for s1 in seq:
        s1.close()
    res["sequential_mlups"] = nodes * steps / (seq_wall_ms * 1e-3) / 1e6
    res["sequential_kernel_ms_per_step"] = ev0.elapsed_time(ev1) / steps
    res["batched_speedup"] = res["mlups"] / res["sequential_mlups"]
    return res


def copy_ceiling(lb, torch, nbytes=2 << 30):
    """Read + write GB/s of the library's streaming copy kernel over 2 GiB."""
    from paper_1701_03637_amd.lbsc import stream_copy
    src = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    stream_copy(dst, src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        stream_copy(dst, src)
    ev1.record()
    torch.cuda.synchronize()
    gbps = 2 * nbytes * 10 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    return gbps


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def host_copy_GBps(nbytes=1 << 30):
    """Read + write GB/s of a numpy copy of 1 GiB (one thread)."""
    import numpy as np
    src = np.ones(nbytes // 8)
    dst = np.empty_like(src)
    np.copyto(dst, src)
    t0 = time.perf_counter()
    for _ in range(3):
        np.copyto(dst, src)
    dt = time.perf_counter() - t0
    return 2 * nbytes * 3 / dt / 1e9


def cpu_baseline(w, steps, steps_one):
    """The FP64 oracle, as it stands, on the host cores, over a bounded sample
    of the headline workload: the same droplet scaled to 256^3 (the 512^3
    lattice would need 160 GB of host memory for the oracle's two FP64
    population sets), timed on all threads and on one."""
    import lbinputs as li
    from oracle.oracle import PSI_RHO, SINK_FACES, Oracle, OracleParams, num_threads, set_num_threads
    n = 256
    ws = li.Workload(f"droplet_{n}^3 (the 512^3 droplet scaled by 1/2)", n, n, n, steps, w.g, w.psi, w.sink,
                     w.rho_h, w.wall_z, "droplet", dict(radius=w.init_args["radius"] * n / w.nx))
    o = Oracle(OracleParams(n, n, n, g=w.g, psi=PSI_RHO, sink=SINK_FACES, rho_h=w.rho_h))
    a, b = ws.densities()
    o.init_from_density(a, b)
    del a, b
    threads = num_threads()
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    set_num_threads(1)
    t1 = time.perf_counter()
    o.step(steps_one)
    dt1 = time.perf_counter() - t1
    set_num_threads(threads)
    return {"value": ws.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{ws.name}, FP64 oracle, {steps} steps on {threads} threads after 1 untimed step "
                      f"({dt:.1f} s); per-node work as the 512^3 headline",
            "one_core_MLUPS": ws.nodes * steps_one / dt1 / 1e6,
            "one_core_sample": f"{steps_one} steps on 1 thread ({dt1:.1f} s)",
            "host_cpu": host_info(), "host_logical_cpus": os.cpu_count(),
            "host_copy_GBps_1thread": host_copy_GBps(),
            "oracle_bytes_per_LU": 2 * 19 * 8 * 4 + 4 * 8,
            }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000, help="timed steps of the headline (512^3) workload")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--forms", default="droplet128,large_fp64,large_fp16n,batched,film",
                    help="extra forms besides the headline (comma list, or 'none')")
    ap.add_argument("--form-steps", type=int, default=400, help="timed steps of each 2M-node form")
    ap.add_argument("--acc-steps", type=int, default=1000,
                    help="steps of the accuracy comparison on 128^3 (0: skipped, profiling aid)")
    ap.add_argument("--d128-precisions", default="fp32s,fp64,fp16n,fp16nf,fp16s",
                    help="storage forms of the 128^3 droplet form (profiling aid: a subset)")
    ap.add_argument("--graph", type=int, default=0, help="steps per HIP graph of the single-lattice forms "
                                                         "(0: direct launches)")
    ap.add_argument("--batch-graph", type=int, default=10, help="steps per HIP graph of the batch (0: direct)")
    ap.add_argument("--tiles", default="",
                    help="pin the headline schedule as nt,tw,th,nzc,variant (skips its tuner)")
    ap.add_argument("--tune-steps", type=int, default=5, help="steps per candidate of the tile tuner (0: defaults)")
    ap.add_argument("--tune-headline", action="store_true",
                    help="tune the headline's schedule too (by default it runs the library's default schedule, "
                         "the one its committed profile was taken on; the tuner's picks at 512^3 are within 1 %%)")
    ap.add_argument("--cpu-steps", type=int, default=15)
    ap.add_argument("--cpu-steps-one", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-headline", action="store_true",
                    help="profiling aid: skip the headline and print the forms alone (not a benchmark line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library steps one GPU; --gpus must be 1 (multi-GPU sharding is a design "
              "note, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import lbinputs as li
    import paper_1701_03637_amd as lb
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lb.load_library()
    forms = [f for f in args.forms.split(",") if f and f != "none"]

    w = li.droplet_512()
    pin = tuple(int(v) for v in args.tiles.split(",")) if args.tiles else None
    if pin is not None and len(pin) != 5:
        sys.exit("--tiles needs five integers: nt,tw,th,nzc,variant")
    head = None
    if not args.no_headline:
        head, sim = form_single(lb, torch, w, "fp32s", args.steps, args.warmup, args.diag_every, args.graph,
                                args.tune_steps if args.tune_headline else 0, pin)
        sim.close()
        torch.cuda.empty_cache()
        print(f"# headline {w.name} fp32s {head['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    extra = {}
    fs = max(args.form_steps // 8, 20)   # 512^3 forms
    if "large_fp64" in forms or "large_fp16n" in forms:
        large = {}
        for prec, key in (("fp64", "large_fp64"), ("fp16n", "large_fp16n")):
            if key not in forms:
                continue
            r, s = form_single(lb, torch, w, prec, fs, 5, 0, args.graph, 0)
            s.close()
            large[prec] = r
            torch.cuda.empty_cache()
            print(f"# {w.name} {prec} {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        acc = accuracy_runs(lb, torch, w, ["fp32s"] + (["fp16n"] if "fp16n" in large else []), fs)
        large["accuracy"] = acc
        if head is not None:
            speedup_at_matched_accuracy(head, large.get("fp64"), acc)
        if "fp16n" in large:
            speedup_at_matched_accuracy(large["fp16n"], large.get("fp64"), acc)
        extra["large"] = large
    if "droplet128" in forms:
        w2 = li.droplet_128()
        d128 = {}
        for prec in args.d128_precisions.split(","):
            r, s = form_single(lb, torch, w2, prec, args.form_steps, 20, args.diag_every, args.graph,
                               args.tune_steps)
            s.close()
            d128[prec] = r
            print(f"# {w2.name} {prec} {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        if args.acc_steps > 0:
            reduced = [p for p in ("fp32s", "fp16n", "fp16nf", "fp16s") if p in d128]
            acc = accuracy_runs(lb, torch, w2, reduced, args.acc_steps)
            d128["accuracy"] = acc
            for prec in reduced:
                speedup_at_matched_accuracy(d128[prec], d128.get("fp64"), acc)
        extra["droplet128"] = d128
        torch.cuda.empty_cache()
    if "batched" in forms:
        extra["batched"] = form_batched(lb, torch, max(args.form_steps // 4, 20), 20, args.batch_graph,
                                        min(args.tune_steps, 5))
        print(f"# batched {extra['batched']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "film" in forms:
        # the film configurations: 64x64x512 (FP32S, FP64, FP16N) and 4x4x128
        # (FP64, its full 1000 steps); walled, sink on the top plane
        films = {}
        for wl, prec, steps in ((li.film_deep(), "fp32s", args.form_steps), (li.film_deep(), "fp64", args.form_steps),
                                (li.film_deep(), "fp16n", args.form_steps),
                                (li.film_small(), "fp64", li.film_small().steps)):
            r, s = form_single(lb, torch, wl, prec, steps, 20, args.diag_every, args.graph, min(args.tune_steps, 5))
            s.close()
            films[f"{wl.name}_{prec}"] = r
            print(f"# film {wl.name} {prec} {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        extra["films"] = films
        torch.cuda.empty_cache()
    ceiling = copy_ceiling(lb, torch)
    if head is None:
        print(json.dumps({"forms": extra, "copy_ceiling_GBps": ceiling}), flush=True)
        return

    kms = head["kernel_ms_per_step"]
    alg_bytes = w.nodes * BYTES_PER_LU["fp32s"]
    achieved = alg_bytes / (kms * 1e-3) / 1e9
    traffic = measured_traffic("droplet512", "fp32s")
    line = {
        "metric": METRIC,
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE["fp32s"],
        "data": "synthetic",
        "config": {"workload": "droplet_512^3 radius 120, psi=rho, g=0.9, tau=1, sink rho_H=0.04 on 6 faces, "
                               "FP32-shifted storage (rho0 = 0.04, 0.70), FP64 diagnostics every "
                               f"{args.diag_every} steps", "nodes": w.nodes, "precision": "fp32s",
                   "graph_steps": args.graph, "tiles": head["tiles"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "kernel": step_kernel_name(head["tiles"]), "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": kms,
                     "frac_wall": alg_bytes / (head["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                     "frac_wall_note": "same bytes over the wall-clock step time (diagnostics included)"},
        "copy_ceiling_GBps": ceiling,
        "headline": head,
        "forms": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps, args.cpu_steps_one)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
