"""Benchmark of the two-component D3Q19 Shan-Chen evaporation step on one MI355X.

Headline: 128^3 droplet (radius 24, psi = rho, g = 0.9, tau = 1, sink
rho_H = 0.04 on all six faces) in FP32-shifted storage, MLUPS over the timed
steps (one step = the fused pull/sink/moments/force/collision/store launch;
FP64 diagnostics every --diag-every steps are inside the timed region).
Extra forms on the same line: plain FP64 and FP16-shifted on the same
workload (with their errors against the FP64 GPU run), 64 batched uneven
droplets (48^3..156^3) in one launch per step, and the 512^3 droplet.

Prints one JSON line. Synthetic inputs only (see lbinputs).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "2-comp D3Q19 MLUPS + % HBM peak; FP32/FP16/batched vs plain FP64 at stated error"
HBM_PEAK_GBPS = 8000.0
# 2 comps x 19 x (read + write) x element size; FP16N stores the rest
# population in FP32 (2 x 2 x (18 x 2 + 4))
BYTES_PER_LU = {"fp64": 608, "fp32s": 304, "fp16s": 152, "fp16n": 160}
DTYPE = {"fp64": "f64", "fp32s": "f32", "fp16s": "f32", "fp16n": "f32"}


def kernel_hash() -> str:
    """Hash of the kernel sources' code: comments and whitespace are dropped,
    so a counter record stays valid across edits that change no code."""
    h = hashlib.sha256()
    for f in ("kernels.h", "lattice.h", "lbsc.hip"):
        with open(os.path.join(ROOT, "paper_1701_03637_amd", "csrc", f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def step_kernel_name(tiles) -> str:
    """Name of the FP32S step kernel a resolved schedule (nt, tw, th, nzc,
    variant) launches."""
    nt, variant = tiles[0], tiles[4]
    if variant == 3:
        return f"lbsc::k_step_pipe<lbsc::StF32S, {nt}>"
    return f"lbsc::k_step<lbsc::StF32S, {nt}, {'false' if variant == 2 else 'true'}>"


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


def make_sim(lb, w, precision, shift=(0.04, 0.70)):
    p = lb.make_params(w.nx, w.ny, w.nz, wall_z=w.wall_z, g=w.g, psi=w.psi, precision=precision, shift=shift,
                       sink=w.sink, rho_h=w.rho_h, sink_radius=w.sink_radius, phi_delta=w.phi_delta)
    return lb.Sim(p)


def timed_run(sim, steps, warmup, diag_every, torch):
    """Warm up, then time `steps` steps with events around each step batch.
    Returns (wall_ms_region, kernel_ms_total, diag)."""
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
    sim = make_sim(lb, w, precision)
    a, b = w.densities()
    if pin:
        sim.set_tiles(*pin)
    elif tune_steps:
        # the tuner advances the state, so initialise again afterwards
        sim.init_from_density(a, b)
        sim.tune(tune_steps)
    sim.init_from_density(a, b)
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
    rho = sim.density(0)
    sim.close()
    return out, rho


def form_batched(lb, torch, steps, warmup, diag_every, tune_steps):
    import lbinputs as li
    ws = li.batch64()
    params = [lb.make_params(w.nx, w.ny, w.nz, g=w.g, psi=w.psi, precision="fp32s", sink=w.sink, rho_h=w.rho_h)
              for w in ws]
    sim = lb.Sim(params)
    dens = [w.densities() for w in ws]
    if tune_steps:
        for k, (a, b) in enumerate(dens):
            sim.init_from_density(a, b, inst=k)
        sim.tune(tune_steps)
    for k, (a, b) in enumerate(dens):
        sim.init_from_density(a, b, inst=k)
    nodes = sum(w.nodes for w in ws)
    m0 = []
    for k in range(len(ws)):
        d = sim.diagnostics(inst=k)
        m0.append((d["mass"][0], d["mass"][0] + d["mass"][1]))
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
        "nodes": nodes, "steps": steps, "mlups": nodes * steps / (wall_ms * 1e-3) / 1e6,
        "kernel_ms_per_step": step_ms / steps,
        "alg_GBps": nodes * 304 / (step_ms / steps * 1e-3) / 1e9,
        "items_per_step": sim.num_items(),
        "tiles": list(sim.tiles()),
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


def cpu_baseline(w, steps):
    """The FP64 oracle, as it stands, on the host cores, over a bounded sample."""
    from oracle.oracle import PSI_RHO, SINK_FACES, Oracle, OracleParams, num_threads
    o = Oracle(OracleParams(w.nx, w.ny, w.nz, g=w.g, psi=PSI_RHO, sink=SINK_FACES, rho_h=w.rho_h))
    a, b = w.densities()
    o.init_from_density(a, b)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return {"value": w.nodes * steps / dt / 1e6, "unit": "MLUPS", "cores": num_threads(), "kind": "oracle",
            "sample": f"{w.name} FP64 oracle, {steps} steps after 1 untimed step ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000, help="timed steps of the headline workload")
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--forms", default="fp64,fp16s,fp16n,batched,large,film",
                    help="extra forms besides the fp32s headline (comma list, or 'none')")
    ap.add_argument("--graph", type=int, default=0, help="steps per HIP graph (0: direct launches)")
    ap.add_argument("--tiles", default="",
                    help="pin the headline schedule as nt,tw,th,nzc,variant (skips its tuner)")
    ap.add_argument("--tune-steps", type=int, default=20, help="steps per candidate of the tile tuner (0: defaults)")
    ap.add_argument("--cpu-steps", type=int, default=120)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    w = li.droplet_128()
    pin = tuple(int(v) for v in args.tiles.split(",")) if args.tiles else None
    if pin is not None and len(pin) != 5:
        sys.exit("--tiles needs five integers: nt,tw,th,nzc,variant")
    head, rho32 = form_single(lb, torch, w, "fp32s", args.steps, args.warmup, args.diag_every, args.graph,
                              args.tune_steps, pin)
    print(f"# fp32s {head['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    extra = {}
    rho64 = None
    if "fp64" in forms:
        f64, rho64 = form_single(lb, torch, w, "fp64", args.steps, args.warmup, args.diag_every, args.graph,
                                 args.tune_steps)
        head["max_abs_drho_vs_fp64"] = float((rho32 - rho64).abs().max())
        head["speedup_vs_fp64"] = head["mlups"] / f64["mlups"]
        extra["fp64"] = f64
        print(f"# fp64 {f64['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    for prec in ("fp16s", "fp16n"):
        if prec not in forms:
            continue
        r, rho = form_single(lb, torch, w, prec, args.steps, args.warmup, args.diag_every, args.graph,
                             args.tune_steps)
        if rho64 is not None:
            r["max_abs_drho_vs_fp64"] = float((rho - rho64).abs().max())
            r["speedup_vs_fp64"] = r["mlups"] / f64["mlups"]
        extra[prec] = r
        del rho
        print(f"# {prec} {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    del rho64
    del rho32
    torch.cuda.empty_cache()
    if "batched" in forms:
        extra["batched"] = form_batched(lb, torch, max(args.steps // 20, 10), 20, args.diag_every,
                                        min(args.tune_steps, 5))
        print(f"# batched {extra['batched']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "large" in forms:
        wl = li.droplet_512()
        big, rho = form_single(lb, torch, wl, "fp32s", max(args.steps // 40, 10), 20, 0, args.graph,
                               min(args.tune_steps, 5))
        del rho
        extra["large"] = big
        print(f"# large {big['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if "film" in forms:
        # the film configurations: 64x64x512 (FP32S and FP64) and 4x4x128
        # (FP64, its full 1000 steps); walled, sink on the top plane
        films = {}
        for wl, prec, steps in ((li.film_deep(), "fp32s", max(args.steps // 10, 10)),
                                (li.film_deep(), "fp64", max(args.steps // 10, 10)),
                                (li.film_small(), "fp64", li.film_small().steps)):
            r, rho = form_single(lb, torch, wl, prec, steps, 20, args.diag_every, args.graph,
                                 min(args.tune_steps, 5))
            del rho
            films[f"{wl.name}_{prec}"] = r
            print(f"# film {wl.name} {prec} {r['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
        extra["films"] = films
        torch.cuda.empty_cache()
    ceiling = copy_ceiling(lb, torch)

    kms = head["kernel_ms_per_step"]
    achieved = w.nodes * BYTES_PER_LU["fp32s"] / (kms * 1e-3) / 1e9
    traffic = measured_traffic("droplet128", "fp32s")
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
        "config": {"workload": "droplet_128^3 radius 24, psi=rho, g=0.9, tau=1, sink rho_H=0.04 on 6 faces, "
                               "FP32-shifted storage (rho0 = 0.04, 0.70), FP64 diagnostics every "
                               f"{args.diag_every} steps", "nodes": w.nodes, "precision": "fp32s",
                   "graph_steps": args.graph, "tiles": head["tiles"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "kernel": step_kernel_name(head["tiles"]), "alg_bytes_per_launch": w.nodes * BYTES_PER_LU["fp32s"],
                     "avg_launch_ms": kms},
        "copy_ceiling_GBps": ceiling,
        "headline": head,
        "forms": extra,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
