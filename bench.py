"""Benchmark of the two-component D2Q9 Shan-Chen step on one MI355X.

One step = the whole hot path over the lattice once: pull-streaming with
periodic x and bounce-back walls, densities and Shan-Chen + buoyancy forces,
velocity-shift BGK collision, store.  Headline workload: the 10000 x 5000
Rayleigh-Taylor lattice (tau = 1, G = 1.5, g = 1e-5, 32 seeded interface
modes), FP64 storage and arithmetic, populations resident in HBM, 100-step
chunks replayed from HIP graphs.  The library times its two passes at
initialisation and runs the fastest per step: one step per kernel pass
(k_step), two steps fused in registers (k_step2, populations cross HBM
once per two steps), or, in the storage modes with FP32 arithmetic, three
(k_step3).

Prints one JSON line: million lattice updates per second (MLUPS; one update
= both components at one site for one step), the HBM roofline of the kernel
that ran, the single-step pass on the same lattice, the FP64 CPU oracle timed
on a bounded sample of the same workload, the reduced-precision storage
modes, and the 16-member batched ensemble (4 x 1024x512, 8 x 2048x1024,
4 x 4096x2048, FP32).

Besides the rates, the line carries the measurements that qualify them:
the density-field error of FP32 storage against FP64 on the headline
lattice at step 2000; mass drift, mixing-width and density errors of the
reduced-precision codes on the 4096 x 2048 lattices (miscible and
immiscible) over 20000 steps against FP64; the 16 ensemble members' errors
against their FP64 runs and the ensemble means of the mixing width and the
energy budget; the 2048 x 1024 lattice's rate under both forcing schemes;
and a plain device copy timed in the same process as a measured roofline
denominator.

    python bench.py [--steps K] [--warmup W] [--storage f64|f32|f16s|bf16s] [--spp 0|1|2|3]
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
# 2 components x 9 populations x (read + write) x element size, plus in the
# 16-bit modes the two FP32 site densities (read + write): the bytes one
# kernel pass moves per site (per lattice update for single steps)
BYTES_PER_LU = {"f64": 288, "f32": 144, "f16s": 88, "bf16s": 88}
KERNEL = {1: "step", 2: "step2", 3: "step3"}
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


def measured_sq(kernel: str, storage: str):
    """Shader-sequencer shares of the kernel (VALU busy, cycles issuing,
    cycles waiting on a dependency) from the committed counter summary, if
    taken from the current kernel sources; else None."""
    from paper_2101_04847_amd.profiling import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "sq_counters_10000x5000.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh)
    for rec in recs:
        if rec.get("kernel") == kernel and rec.get("storage") == storage and rec.get("source_hash") == kernel_source_hash():
            return {k: rec[k] for k in ("valu_busy", "issue_any", "wait_dependency", "tile")}
    return None


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def kernel_launch_ms(lat, spp: int, stream, n: int = 12) -> float:
    """Average duration of one pass of spp steps (one kernel launch), timed
    with events on `stream` around n eager lb_step(spp) calls after one
    untimed call."""
    import torch

    lat.step(spp)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(n):
        lat.step(spp)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / n


def graph_chunk_for(steps: int) -> int:
    """Steps per captured graph: 100, or the whole (even) timed run when it
    is shorter, so that the timed region replays at least one graph."""
    return 100 if steps >= 100 else max(2, steps - steps % 2)


def copy_bandwidth(stream, gbytes: float = 4.0, reps: int = 5) -> dict:
    """Best plain device-to-device copy (read + write of gbytes each way) over
    the probe's copy variants and grid sizes, timed with events on `stream`
    in this process (libbwprobe.so)."""
    import ctypes

    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2101_04847_amd", "libbwprobe.so"))
    lib.bw_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                            ctypes.c_void_p]
    lib.bw_copy.restype = ctypes.c_int
    n = int(gbytes * 1e9) // 4096 * 4096
    a = torch.zeros(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    sp = ctypes.c_void_p(stream.cuda_stream)
    results = []
    for v in range(lib.bw_copy_variants()):
        for grid in (2048, 8192, 32768, 65536):
            def run():
                rc = lib.bw_copy(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, v, grid, sp)
                if rc != 0:
                    raise RuntimeError(f"bw_copy variant {v} grid {grid}: status {rc}")
            run()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                run()
            e1.record(stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / reps
            results.append({"variant": v, "grid": grid, "GBs": round(2 * n / (ms / 1e3) / 1e9, 1)})
    del a, b
    torch.cuda.empty_cache()
    best = max(results, key=lambda r: r["GBs"])
    return {"GBs": best["GBs"], "variant": best["variant"], "grid": best["grid"], "bytes_each_way": n,
            "kernel": "bw_copy (paper_2101_04847_amd/csrc/bw_probe.hip)", "candidates": len(results)}


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


def hbm_frac_single_step_basis(storage, ms_step, sites):
    """Fraction of the published HBM bandwidth that the single-step method's
    bytes (every population read and written once per step) would need at
    this rate; above 1 when two steps share one pass over HBM."""
    return round(BYTES_PER_LU[storage] * sites / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)


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
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
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
           "kernel": "lbk::k_" + KERNEL[got], "tile": list(tile), "bytes_per_lu": round(BYTES_PER_LU[name] / got, 2),
           "hbm_frac": hbm_frac(name, got, ms, sites),
           "hbm_frac_single_step_basis": hbm_frac_single_step_basis(name, ms, sites)}
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


def _rel_l2(a, b) -> float:
    """||a - b|| / ||b|| of two device tensors, in FP64 on the GPU."""
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def fp32_error_line(lb, inputs, stream, steps=2000):
    """The headline lattice advanced `steps` steps with FP64 and with FP32
    storage side by side: relative L2 errors of the density fields, phi and
    |u|, the largest density difference, and the mixing widths."""
    import torch
    wl = inputs.LARGE_10000x5000
    out = {"workload": wl.name, "step": steps}
    fields = {}
    for name in ("f64", "f32"):
        lat = lattice_for(lb, [wl], storage_code(lb, name), stream=stream)
        m0 = lat.diagnostics(0)
        lat.step(steps)
        fields[name] = lat.fields(0)
        d = lat.diagnostics(0)
        out[f"{name}_mass_drift"] = max(abs(d["mass_A"] - m0["mass_A"]) / m0["mass_A"],
                                        abs(d["mass_B"] - m0["mass_B"]) / m0["mass_B"])
        out[f"{name}_mixing_width"] = lat.mixing_width(0)["width"]
        release(lat)
    a, b = fields["f32"], fields["f64"]
    out["rel_l2_rhoA"] = _rel_l2(a["rhoA"], b["rhoA"])
    out["rel_l2_rhoB"] = _rel_l2(a["rhoB"], b["rhoB"])
    out["rel_l2_phi"] = _rel_l2(a["rhoA"] - a["rhoB"], b["rhoA"] - b["rhoB"])
    out["rel_l2_speed"] = _rel_l2(torch.hypot(a["ux"], a["uy"]), torch.hypot(b["ux"], b["uy"]))
    out["max_abs_rho"] = float(max((a["rhoA"] - b["rhoA"]).abs().max(), (a["rhoB"] - b["rhoB"]).abs().max()))
    del fields, a, b
    torch.cuda.empty_cache()
    return out


def _series_run(lb, wl, storage, stream, steps, every):
    """One lattice advanced in graph-replayed chunks of `every` steps: the
    masses and mixing width at every sample, the final densities, and the
    event-timed step rate (samples excluded)."""
    import torch
    lat = lattice_for(lb, [wl], storage, stream=stream, graph_chunk=every)
    mass, width = [], []
    ms = 0.0
    for t in range(0, steps + 1, every):
        if t:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lat.step(every)
            e1.record(stream)
            e1.synchronize()
            ms += e0.elapsed_time(e1)
        d = lat.diagnostics(0, check_finite=False)
        mass.append((d["mass_A"], d["mass_B"]))
        width.append(lat.mixing_width(0)["width"])
    f = lat.fields(0)
    fin = {k: f[k] for k in ("rhoA", "rhoB")}
    spp = lat.steps_per_pass
    release(lat)
    return {"mass": mass, "width": width, "fields": fin, "ms_per_step": ms / steps, "spp": spp,
            "finite": bool(d["finite"])}


def reduced_precision_lines(lb, inputs, stream, steps=20000, every=100):
    """The 4096 x 2048 lattices (miscible G = 0.5 and immiscible G = 1.5):
    FP32, FP16S and BF16S storage against the FP64 run of the same lattice
    over `steps` steps: the largest relative mass drift of either component
    over the run, the mixing-width error (largest over the samples and at
    the end), the final relative L2 density error, and the step rate."""
    import torch
    res = []
    for wl in inputs.PRECISION_4096x2048:
        ref = _series_run(lb, wl, lb.F64, stream, steps, every)
        h64 = ref["width"]
        row = {"workload": wl.name, "G_AB": wl.G, "steps": steps, "every": every,
               "f64": {"MLUPS": round(wl.nx * wl.ny / (ref["ms_per_step"] / 1e3) / 1e6, 1),
                       "mass_drift": _drift(ref["mass"]), "mixing_width_final": h64[-1]}}
        for name in ("f32", "f16s", "bf16s"):
            r = _series_run(lb, wl, storage_code(lb, name), stream, steps, every)
            h = r["width"]
            row[name] = {
                "MLUPS": round(wl.nx * wl.ny / (r["ms_per_step"] / 1e3) / 1e6, 1), "steps_per_pass": r["spp"],
                "mass_drift": _drift(r["mass"]),
                "mixing_width_final": h[-1],
                "mixing_width_rel_err_final": abs(h[-1] - h64[-1]) / abs(h64[-1]),
                "mixing_width_max_abs_err": max(abs(x - y) for x, y in zip(h, h64)),
                "rel_l2_rhoA_final": _rel_l2(r["fields"]["rhoA"], ref["fields"]["rhoA"]),
                "rel_l2_rhoB_final": _rel_l2(r["fields"]["rhoB"], ref["fields"]["rhoB"]),
                "finite": r["finite"]}
            del r
            torch.cuda.empty_cache()
        del ref
        torch.cuda.empty_cache()
        res.append(row)
    return res


def _drift(mass) -> float:
    """Largest |M_s(t) - M_s(0)| / M_s(0) over the samples and both components."""
    return max(abs(m[s] - mass[0][s]) / mass[0][s] for m in mass for s in (0, 1))


def ensemble_error_line(lb, inputs, stream, steps=1000):
    """The 16-member ensemble advanced `steps` steps in FP32 and in FP64 (one
    launch per pass over all members each): per member the relative L2
    errors of the density fields of FP32 against FP64; ensemble means and
    spreads (per coupling) of the mixing width and the energy-budget terms of
    the FP32 run."""
    import torch
    wls = inputs.ensemble_16()
    runs = {}
    for name in ("f64", "f32"):
        lat = lattice_for(lb, wls, storage_code(lb, name), stream=stream)
        lat.step(steps)
        per = []
        for k in range(len(wls)):
            f = lat.fields(k)
            d = lat.diagnostics(k)
            b = lat.energy_budget(k)
            per.append({"rhoA": f["rhoA"], "rhoB": f["rhoB"], "width": lat.mixing_width(k)["width"],
                        "Ek": d["Ek"], "Ep": d["Ep"], "buoyancy": d["buoyancy"],
                        **{q: b[q] for q in ("pb", "korteweg", "ktau", "viscous")}})
        runs[name] = per
        release(lat)
    errs = []
    for k, wl in enumerate(wls):
        a, b = runs["f32"][k], runs["f64"][k]
        errs.append({"member": k, "nx": wl.nx, "ny": wl.ny, "G_AB": wl.G,
                     "rel_l2_rho": max(_rel_l2(a["rhoA"], b["rhoA"]), _rel_l2(a["rhoB"], b["rhoB"])),
                     "width_rel_err": abs(a["width"] - b["width"]) / abs(b["width"])})
    groups = {}
    import statistics
    for G in sorted({wl.G for wl in wls}):
        idx = [k for k, wl in enumerate(wls) if wl.G == G]
        grp = {}
        for q in ("width", "Ek", "Ep", "buoyancy", "pb", "korteweg", "ktau", "viscous"):
            v = [runs["f32"][k][q] for k in idx]
            grp[q] = {"mean": statistics.fmean(v), "std": statistics.pstdev(v)}
        groups[f"G={G}"] = grp
    del runs
    torch.cuda.empty_cache()
    return {"step": steps, "storage": "f32 vs f64",
            "rel_l2_rho_max": max(e["rel_l2_rho"] for e in errs),
            "rel_l2_rho_mean": statistics.fmean(e["rel_l2_rho"] for e in errs),
            "width_rel_err_max": max(e["width_rel_err"] for e in errs),
            "members": errs, "ensemble_means_f32": groups}


def medium_lines(lb, inputs, stream, steps=1000, warmup=100):
    """The 2048 x 1024 lattice (FP64) under both forcing schemes: step rate
    and pass chosen."""
    out = []
    wl = inputs.MEDIUM_2048x1024
    rA, rB = wl.densities()
    for name, forcing in (("velocity-shift", lb.FORCE_SHIFT), ("guo", lb.FORCE_GUO)):
        m = lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity)
        lat = lb.Lattice([m], forcing=forcing, storage=lb.F64, graph_chunk=100, stream=stream)
        ms, _ = time_steps(lat, steps, warmup, stream)
        spp, tile = lat.steps_per_pass, lat.tile_shape()
        release(lat)
        out.append({"workload": wl.name, "forcing": name, "storage": "f64",
                    "MLUPS": round(wl.nx * wl.ny / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms, 4),
                    "steps_per_pass": spp, "tile": list(tile),
                    "hbm_frac": hbm_frac("f64", spp, ms, wl.nx * wl.ny)})
    return out


def parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f64", choices=sorted(BYTES_PER_LU))
    ap.add_argument("--tile", default="", help="TXxH, e.g. 256x16 (default: timed choice)")
    ap.add_argument("--spp", type=int, default=0, choices=(0, 1, 2, 3),
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
    chunk = graph_chunk_for(args.steps)
    t_init = time.perf_counter()
    lat = lattice_for(lb, [wl], storage_code(lb, args.storage), tile=tile, stream=stream, spp=args.spp,
                      graph_chunk=chunk)
    t_init = time.perf_counter() - t_init
    tx, th = lat.tile_shape()
    spp = lat.steps_per_pass
    log(f"{wl.name} storage={args.storage} steps/pass={spp} tile={tx}x{th} warmup={args.warmup} steps={args.steps}"
        f" graph chunk={chunk}")
    # the warm-up leaves the buffer parity and graph alignment of the timed
    # region as they are; lb_step replays one graph per full chunk of a call
    chunk_ms = []
    ms_step, wall = time_steps(lat, args.steps, args.warmup, stream, chunk=chunk, chunks_out=chunk_ms)
    replays = (args.steps // chunk) if args.steps >= chunk else 0
    eager_steps = args.steps - replays * chunk
    d = lat.diagnostics(0)
    # the dominant kernel's own launch duration: events around eager passes
    # of spp steps each (one launch per lb_step call shorter than a graph
    # chunk) on the lattice's stream, right after the timed region (the
    # timed region's chunks also hold the passes that take a remainder of a
    # chunk, e.g. one single step per 100 steps with three-step passes)
    launch_ms = kernel_launch_ms(lat, spp, stream) if spp < chunk else ms_step * spp
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
    alg_bytes = BYTES_PER_LU[args.storage] * sites
    achieved = alg_bytes / (launch_ms / 1e3) / 1e9
    traffic = measured_traffic(kernel, args.storage, wl.nx, wl.ny, tile=[tx, th])
    log("measured copy bandwidth")
    copy = copy_bandwidth(stream)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_launch": alg_bytes, "bytes_per_lu": round(BYTES_PER_LU[args.storage] / spp, 2),
            "kernel": "lbk::k_" + kernel, "steps_per_launch": spp, "launch_ms": round(launch_ms, 4),
            # counted HBM-side bytes over the algorithmic bytes of one launch
            "traffic_over_algorithmic": None if traffic is None else round(traffic / alg_bytes, 3),
            # the single-step method's bytes per update (every population
            # read and written once per step) at this rate: above the HBM
            # peak when two steps share one pass over the populations
            "effective_GBs": round(mlups * 1e6 * BYTES_PER_LU[args.storage] / 1e9, 1),
            "frac_single_step_basis": hbm_frac_single_step_basis(args.storage, ms_step, sites),
            "frac_basis_note": ("frac counts the launch's own bytes (each population read and written once "
                                f"per launch of {spp} step(s)); frac_single_step_basis counts "
                                f"{BYTES_PER_LU[args.storage]} B per update, which fused steps need not move"),
            # what limits the kernel, from its committed shader-sequencer counters
            # (profiles/sq_counters_10000x5000.md): a memory-bound pass waits on
            # loads; the one-wave-per-SIMD three-step pass issues in most cycles
            "sq_counters": measured_sq(kernel, args.storage),
            # a plain device copy of 4 GB each way, timed in this process
            "measured_copy_GBs": copy["GBs"], "frac_of_measured_copy": round(achieved / copy["GBs"], 4),
            "measured_copy": copy}

    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "tau": wl.tau, "G_AB": wl.G, "g": wl.g,
                   "forcing": "velocity-shift", "storage": args.storage, "steps_per_pass": spp,
                   "tile": [tx, th], "graph_chunk": chunk, "graph_replays_timed": replays,
                   "eager_steps_timed": eager_steps, "lb_init_s": round(t_init, 3), "wall_s": round(wall, 3)},
        "roofline": roof,
        "state_check": {"finite": d["finite"], "umax": d["umax"], "t": d["t"]},
        # ms per step of each chunk (one graph replay) inside the timed region
        "chunk_ms_per_step": {"median": round(float(sorted(chunk_ms)[len(chunk_ms) // 2]), 4),
                              "min": round(min(chunk_ms), 4), "max": round(max(chunk_ms), 4), "n": len(chunk_ms)},
        "analysis_ms": {"diagnostics": round(min(t_diag) * 1e3, 3), "energy_budget": round(min(t_budget) * 1e3, 3),
                        "interface_length": round(min(t_iface) * 1e3, 3), "components": round(min(t_comp) * 1e3, 3),
                        "budget": {k: budget[k] for k in ("pb", "korteweg", "ktau", "viscous", "buoyancy")},
                        "interface": {"length": iface["length"], "components_A": comps["A"],
                                      "components_B": comps["B"]}},
    }
    if not args.no_extras:
        if spp >= 2:
            log("single-step pass")
            out["single_step"] = variant_line(lb, inputs, args.storage, stream, spp=1)
        if spp == 3:
            log("two-step pass")
            out["two_step"] = variant_line(lb, inputs, args.storage, stream, spp=2)
        out["storage_variants"] = []
        for name in ("f32", "f16s", "bf16s"):
            if name != args.storage:
                log("storage variant", name)
                out["storage_variants"].append(variant_line(lb, inputs, name, stream))
        log("FP32 against FP64 at step 2000")
        out["fp32_error_10000x5000"] = fp32_error_line(lb, inputs, stream)
        log("reduced precision on 4096x2048, 20000 steps")
        out["reduced_precision_4096x2048"] = reduced_precision_lines(lb, inputs, stream)
        log("ensemble of 16")
        out["ensemble"] = ensemble_line(lb, inputs, stream)
        log("ensemble errors")
        out["ensemble"]["errors"] = ensemble_error_line(lb, inputs, stream)
        log("2048x1024, both forcings")
        out["medium_2048x1024"] = medium_lines(lb, inputs, stream)
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
