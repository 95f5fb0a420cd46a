"""Benchmark of the two-component D2Q9 Shan-Chen step on one MI355X.

One step = the whole hot path over the lattice once: pull-streaming with
periodic x and bounce-back walls, densities and Shan-Chen + buoyancy forces,
velocity-shift BGK collision, store.  Headline workload: the 10000 x 5000
Rayleigh-Taylor lattice (tau = 1, G = 1.5, g = 1e-5, 32 seeded interface
modes), FP64 storage and arithmetic, populations resident in HBM, 100-step
chunks replayed from HIP graphs.  The library times its two passes at
initialisation and runs the faster per step: one step per kernel pass
(k_step), or two steps fused in registers (k_step2, populations cross HBM
once per two steps).

Prints one JSON line: million lattice updates per second (MLUPS; one update
= both components at one site for one step), the HBM roofline of the kernel
that ran, the single-step pass on the same lattice, the FP64 CPU oracle timed
on a bounded sample of the same workload, the reduced-precision storage
modes, and the 16-member batched ensemble (4 x 1024x512, 8 x 2048x1024,
4 x 4096x2048, FP32).

    python bench.py [--steps K] [--warmup W] [--storage f64|f32|f16s|bf16s] [--spp 0|1|2]
    python bench.py --report out.json     # precision and ensemble studies
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# 2 components x 9 populations x (read + write) x element size: the bytes
# one kernel pass moves per site (per lattice update for single steps)
BYTES_PER_LU = {"f64": 288, "f32": 144, "f16s": 72, "bf16s": 72}
KERNEL = {1: "step", 2: "step2"}
METRIC = "MLUPS + % HBM peak, 2-comp D2Q9 Shan-Chen 10000×5000; ensemble MLUPS"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str, storage: str, nx: int, ny: int, tile=None):
    """HBM bytes per launch of the kernel from the committed counter summary,
    if it was taken from the current kernel sources and, when the record
    names one, with the same tile; else None."""
    from paper_2101_04847_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"{kernel}_{storage}_{nx}x{ny}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh)
    # one record, or a list of records taken at different tiles
    for rec in recs if isinstance(recs, list) else [recs]:
        if rec.get("source_hash") != kernel_source_hash():
            continue
        if tile is not None and rec.get("tile") is not None and list(rec["tile"]) != list(tile):
            continue
        return rec.get("bytes_per_launch")
    return None


def storage_code(lb, name):
    return {"f64": lb.F64, "f32": lb.F32, "f16s": lb.F16S, "bf16s": lb.BF16S}[name]


def lattice_for(lb, workloads, storage, tile=(0, 0), stream=None, graph_chunk=100, spp=0, **walls):
    members = []
    for wl in workloads:
        rA, rB = wl.densities()
        members.append(lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity, **walls))
    return lb.Lattice(members, forcing=lb.FORCE_SHIFT, storage=storage, tile_x=tile[0], tile_h=tile[1],
                      graph_chunk=graph_chunk, stream=stream, steps_per_pass=spp)


def hbm_frac(storage, spp, ms_step, sites):
    """Fraction of the published HBM bandwidth that the pass's own bytes
    (every population read and written once per pass) represent."""
    return round(BYTES_PER_LU[storage] * sites / (ms_step * spp / 1e3) / 1e9 / HBM_PEAK_GBS, 4)


def time_steps(lat, steps, warmup, stream, chunk=100, chunks_out=None):
    """ms per step over `steps` steps, timed with events on the lattice's
    stream after `warmup` untimed steps; plus the host wall time.  Events
    also bracket every `chunk` steps (one graph replay); their per-chunk
    times go to chunks_out when given."""
    import torch
    lat.step(warmup)
    torch.cuda.synchronize()
    n_chunks = max(1, steps // chunk)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_chunks + 1)]
    ev_end = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    evs[0].record(stream)
    done = 0
    for k in range(n_chunks):
        n = chunk if k < n_chunks - 1 else steps - done
        lat.step(n)
        done += n
        evs[k + 1].record(stream)
    ev_end.record(stream)
    torch.cuda.synchronize()
    if chunks_out is not None:
        chunks_out.extend(evs[k].elapsed_time(evs[k + 1]) / (chunk if k < n_chunks - 1 else steps - chunk * k)
                          for k in range(n_chunks))
    return evs[0].elapsed_time(ev_end) / steps, time.perf_counter() - w0


def release(lat):
    import torch
    lat.close()
    del lat
    torch.cuda.empty_cache()


def cpu_baseline(wl, target_s: float = 40.0) -> dict:
    """The FP64 oracle on the host cores: full lattice, a few steps."""
    import oracle
    oracle.build(force=False)
    rA, rB = wl.densities()
    p = oracle.Params(nx=wl.nx, ny=wl.ny, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
    f = oracle.fill_equilibrium(p, rA, rB)
    oracle.run_inplace(p, f, 1)      # first touch of the buffers
    t0 = time.perf_counter()
    oracle.run_inplace(p, f, 1)
    one = time.perf_counter() - t0
    n = max(1, min(30, int(target_s / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.run_inplace(p, f, n)
    dt = time.perf_counter() - t0
    # the same step on one thread (one step of the full lattice)
    cores = oracle.threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.run_inplace(p, f, 1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    del f
    return {"value": round(wl.nx * wl.ny * n / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{n} steps of the full {wl.nx}x{wl.ny} lattice after 2 untimed steps "
                      f"(FP64, OpenMP over rows, {dt:.1f} s)",
            "single_thread": {"value": round(wl.nx * wl.ny / dt1 / 1e6, 3), "unit": "MLUPS",
                              "sample": f"1 further step of the same lattice on one thread ({dt1:.1f} s)"}}


def variant_line(lb, inputs, name, stream, steps=300, warmup=50, spp=0, **walls):
    wl = inputs.LARGE_10000x5000
    lat = lattice_for(lb, [wl], storage_code(lb, name), stream=stream, spp=spp, **walls)
    tile, got = lat.tile_shape(), lat.steps_per_pass
    ms, _ = time_steps(lat, steps, warmup, stream)
    release(lat)
    sites = wl.nx * wl.ny
    mlups = sites / (ms / 1e3) / 1e6
    out = {"storage": name, "MLUPS": round(mlups, 1), "ms_per_step": round(ms, 4), "steps_per_pass": got,
           "kernel": "lbk::k_" + KERNEL[got], "tile": list(tile), "bytes_per_lu": BYTES_PER_LU[name] // got,
           "hbm_frac": hbm_frac(name, got, ms, sites)}
    if walls:
        out["walls"] = {k: list(v) if isinstance(v, tuple) else v for k, v in walls.items()}
    return out


# algorithmic HBM bytes per 3D site update: the density pass reads 38
# populations and writes 2 densities (FP64); the collide pass reads 38
# populations and the densities (each once, the neighbours' from cache) and
# writes 38 populations
BYTES_PER_LU_3D = {"f64": 38 * 8 + 16 + 38 * 8 + 16 + 38 * 8, "f32": 38 * 4 + 16 + 38 * 4 + 16 + 38 * 4}
# the fused pass: every population read once and written once (densities stay in LDS)
BYTES_PER_LU_3D_FUSED = {"f64": 2 * 38 * 8, "f32": 2 * 38 * 4}


def d3q19_line(lb, inputs, stream, storage="f64", steps=100, warmup=10, two_pass=False):
    from paper_2101_04847_amd import lb3
    w = inputs.D3_384
    rA, rB = inputs.rt3d_densities(w["nx"], w["ny"], w["nz"], w["seed"])
    lat = lb3.Lattice3(w["nx"], w["ny"], w["nz"], rA, rB, tau=(w["tau"], w["tau"]), G=w["G"],
                       g=((0.0, -w["g"], 0.0), (0.0, w["g"], 0.0)), storage=storage_code(lb, storage),
                       stream=stream, two_pass=two_pass)
    del rA, rB
    ms, _ = time_steps(lat, steps, warmup, stream, chunk=steps)
    d = lat.diagnostics()
    lat.close()
    del lat
    import torch
    torch.cuda.empty_cache()
    sites = w["nx"] * w["ny"] * w["nz"]
    mlups = sites / (ms / 1e3) / 1e6
    bpl = BYTES_PER_LU_3D[storage] if two_pass else BYTES_PER_LU_3D_FUSED[storage]
    return {"workload": w["name"], "storage": storage, "MLUPS": round(mlups, 1), "ms_per_step": round(ms, 4),
            "kernels": ["lbk3::k3_density", "lbk3::k3_collide"] if two_pass else ["lbk3::k3_fused"],
            "bytes_per_lu": bpl, "hbm_frac": round(bpl * sites / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "finite": d["finite"], "umax": d["umax"]}


def ensemble_line(lb, inputs, stream, storage="f32", steps=300, warmup=50):
    wls = inputs.ensemble_16()
    lat = lattice_for(lb, wls, storage_code(lb, storage), stream=stream)
    tiles = sorted({(wl.nx, wl.ny, *lat.tile_shape(k)) for k, wl in enumerate(wls)})
    got = lat.steps_per_pass
    ms, _ = time_steps(lat, steps, warmup, stream)
    release(lat)
    sites = sum(wl.nx * wl.ny for wl in wls)
    mlups = sites / (ms / 1e3) / 1e6
    return {"members": len(wls), "sites": sites, "storage": storage, "MLUPS": round(mlups, 1),
            "ms_per_step": round(ms, 4), "graph_chunk": 100, "steps_per_pass": got,
            "kernel": "lbk::k_" + KERNEL[got], "hbm_frac": hbm_frac(storage, got, ms, sites),
            "tiles": [list(t) for t in tiles],
            "config": "4x1024x512 + 8x2048x1024 + 4x4096x2048, G alternating 0.5 / 1.5, seeds 100-115"}


def parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f64", choices=sorted(BYTES_PER_LU))
    ap.add_argument("--tile", default="", help="TXxH, e.g. 256x16 (default: timed choice)")
    ap.add_argument("--spp", type=int, default=0, choices=(0, 1, 2),
                    help="steps per kernel pass (0: timed choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the storage variants and the ensemble")
    ap.add_argument("--report", default="", help="run the precision / ensemble studies, write JSON here")
    ap.add_argument("--d3q19-only", action="store_true",
                    help="time only the 3D (D3Q19) step on 384^3 in --storage (for kernel traces)")
    ap.add_argument("--two-pass", action="store_true", help="with --d3q19-only: the two-pass 3D step")
    return ap


def main() -> int:
    args = parser().parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the step shards across GPUs "
              "as described in the design notes, but this implementation runs on a single MI355X.", file=sys.stderr)
        return 2

    import torch

    from paper_2101_04847_amd import inputs, lb

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    if args.d3q19_only:
        if args.storage not in BYTES_PER_LU_3D:
            print("the 3D step stores f64 or f32", file=sys.stderr)
            return 2
        print(json.dumps({"d3q19": d3q19_line(lb, inputs, stream, args.storage, steps=min(args.steps, 200),
                                              warmup=min(args.warmup, 10), two_pass=args.two_pass)}), flush=True)
        return 0
    if args.report:
        from paper_2101_04847_amd import studies
        rep = studies.run_all(lb, inputs, stream, log)
        with open(args.report, "w") as fh:
            json.dump(rep, fh, indent=1)
        print(json.dumps({"report": args.report, "sections": sorted(rep)}), flush=True)
        return 0

    wl = inputs.LARGE_10000x5000
    tile = (0, 0)
    if args.tile:
        a, b = args.tile.lower().split("x")
        tile = (int(a), int(b))
    lat = lattice_for(lb, [wl], storage_code(lb, args.storage), tile=tile, stream=stream, spp=args.spp)
    tx, th = lat.tile_shape()
    spp = lat.steps_per_pass
    log(f"{wl.name} storage={args.storage} steps/pass={spp} tile={tx}x{th} warmup={args.warmup} steps={args.steps}")
    chunk_ms = []
    ms_step, wall = time_steps(lat, args.steps, args.warmup, stream, chunks_out=chunk_ms)
    d = lat.diagnostics(0)
    # cost of the analysis passes (each call synchronises): energy-budget
    # averages and the kinetic-energy balance terms, best of three
    t_diag, t_budget, t_iface, t_comp = [], [], [], []
    for _ in range(3):
        t0 = time.perf_counter()
        lat.diagnostics(0)
        t_diag.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        budget = lat.energy_budget(0)
        t_budget.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        iface = lat.interface_length(0)
        t_iface.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        comps = lat.components(0)
        t_comp.append(time.perf_counter() - t0)
    release(lat)
    sites = wl.nx * wl.ny
    mlups = sites / (ms_step / 1e3) / 1e6

    # roofline of the kernel that ran: one launch per pass of spp steps;
    # algorithmic bytes per launch = 2 components x 9 populations x
    # (read + write) x element size per site, i.e. BYTES_PER_LU / spp per
    # lattice update
    kernel = KERNEL[spp]
    launch_ms = ms_step * spp
    alg_bytes = BYTES_PER_LU[args.storage] * sites
    achieved = alg_bytes / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(kernel, args.storage, wl.nx, wl.ny, tile=[tx, th])
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": alg_bytes, "bytes_per_lu": BYTES_PER_LU[args.storage] // spp,
            "kernel": "lbk::k_" + kernel, "steps_per_launch": spp, "launch_ms": round(launch_ms, 4),
            # the single-step method's 288 B per update at this rate (above
            # the HBM peak when two steps are fused)
            "effective_GBs": round(mlups * 1e6 * BYTES_PER_LU[args.storage] / 1e9, 1)}

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "tau": wl.tau, "G_AB": wl.G, "g": wl.g,
                   "forcing": "velocity-shift", "storage": args.storage, "steps_per_pass": spp,
                   "tile": [tx, th], "graph_chunk": 100, "wall_s": round(wall, 3)},
        "roofline": roof,
        "state_check": {"finite": d["finite"], "umax": d["umax"], "t": d["t"]},
        # ms per step of each 100-step graph replay inside the timed region
        "chunk_ms_per_step": {"median": round(float(sorted(chunk_ms)[len(chunk_ms) // 2]), 4),
                              "min": round(min(chunk_ms), 4), "max": round(max(chunk_ms), 4), "n": len(chunk_ms)},
        "analysis_ms": {"diagnostics": round(min(t_diag) * 1e3, 3), "energy_budget": round(min(t_budget) * 1e3, 3),
                        "interface_length": round(min(t_iface) * 1e3, 3), "components": round(min(t_comp) * 1e3, 3),
                        "budget": {k: budget[k] for k in ("pb", "korteweg", "ktau", "viscous", "buoyancy")},
                        "interface": {"length": iface["length"], "components_A": comps["A"],
                                      "components_B": comps["B"]}},
    }
    if not args.no_extras:
        if spp == 2:
            log("single-step pass")
            out["single_step"] = variant_line(lb, inputs, args.storage, stream, spp=1)
        out["storage_variants"] = []
        for name in ("f32", "f16s", "bf16s"):
            if name != args.storage:
                log("storage variant", name)
                out["storage_variants"].append(variant_line(lb, inputs, name, stream))
        log("ensemble of 16")
        out["ensemble"] = ensemble_line(lb, inputs, stream)
        # wetting walls (Eq. 6 force, psi = 0 on boundary nodes): the wall-term kernels
        log("wetting walls")
        out["wetting_walls"] = variant_line(lb, inputs, args.storage, stream, G_wall=(0.05, -0.05),
                                            wall_psi=lb.PSI_ZERO)
        # the D3Q19 extension on 384^3
        out["d3q19"] = []
        for st, two in (("f64", False), ("f32", False), ("f64", True)):
            log("d3q19", st, "two passes" if two else "fused")
            out["d3q19"].append(d3q19_line(lb, inputs, stream, st, two_pass=two))
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
