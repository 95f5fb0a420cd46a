"""Precision and ensemble studies run through liblb (host-side analysis of the
library's outputs only; every lattice update runs in the HIP kernels).

* fp32_vs_fp64_large: the 10000 x 5000 workload advanced 2000 steps with FP64
  and with FP32 storage; relative L2 error of the density fields.
* reduced_precision: the 4096 x 2048 workload, miscible (G = 0.5) and
  immiscible (G = 1.5), 20000 steps with energy-budget averages every 100
  steps, in FP64 (reference), FP32, FP16S and BF16S; per-component mass
  drift, mixing-width error and final density error against FP64.
* ensemble_statistics: the 16-member ensemble (FP32) for 20000 steps with
  averages every 100 steps; ensemble mean and spread of the mixing width,
  kinetic and potential energy and every term of the kinetic-energy balance
  (Eq. 15-22: bulk pressure, Korteweg and tau stresses, viscous term,
  buoyancy), per coupling, and how well Eq. 17 closes per member.
"""
from __future__ import annotations

import time

import numpy as np

TRIM = 10


def _lattice(lb, wls, storage, stream, rho0=(0.0, 0.0)):
    members = []
    for wl in wls:
        rA, rB = wl.densities()
        members.append(lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity, rho0=rho0))
    return lb.Lattice(members, forcing=lb.FORCE_SHIFT, storage=storage, graph_chunk=100, stream=stream,
                      diag_trim=TRIM)


def _close(lat):
    import torch
    lat.close()
    torch.cuda.empty_cache()


def _rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))


def phi_reference(profile0, trim=TRIM):
    """Half the jump of the row-mean order parameter between the bulk rows
    just inside the trimmed domain at t = 0."""
    p = np.asarray(profile0)
    return 0.5 * abs(p[len(p) - trim - 1] - p[trim])


def fp32_vs_fp64_large(lb, inputs, stream, log, steps=2000):
    wl = inputs.LARGE_10000x5000
    fields = {}
    timing = {}
    for name, st in (("f64", lb.F64), ("f32", lb.F32)):
        log(f"10000x5000 {name}: {steps} steps")
        lat = _lattice(lb, [wl], st, stream)
        t0 = time.perf_counter()
        lat.step(steps)
        f = lat.fields(0)
        fields[name] = {k: f[k].cpu().numpy() for k in ("rhoA", "rhoB", "ux", "uy")}
        timing[name] = time.perf_counter() - t0
        _close(lat)
    ref, lo = fields["f64"], fields["f32"]
    phi_ref = ref["rhoA"] - ref["rhoB"]
    phi_lo = lo["rhoA"] - lo["rhoB"]
    return {
        "workload": wl.name, "steps": steps,
        "rel_l2_rhoA": _rel_l2(lo["rhoA"], ref["rhoA"]),
        "rel_l2_rhoB": _rel_l2(lo["rhoB"], ref["rhoB"]),
        "rel_l2_phi": _rel_l2(phi_lo, phi_ref),
        "max_abs_rho": float(max(np.max(np.abs(lo["rhoA"] - ref["rhoA"])), np.max(np.abs(lo["rhoB"] - ref["rhoB"])))),
        "rel_l2_u": _rel_l2(np.hypot(lo["ux"], lo["uy"]), np.hypot(ref["ux"], ref["uy"])),
        "wall_s": {k: round(v, 2) for k, v in timing.items()},
    }


BUDGET_KEYS = ("pb", "korteweg", "ktau", "viscous")


def _series(lb, wls, storage, stream, steps, every, log, tag, rho0=(0.0, 0.0), budget=False):
    lat = _lattice(lb, wls, storage, stream, rho0)
    n = len(wls)
    keys = ["t", "mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "h"] + (list(BUDGET_KEYS) if budget else [])
    out = [{k: [] for k in keys} for _ in range(n)]
    phi_refs = []
    for m in range(n):
        d = lat.diagnostics(m, profile=True)
        phi_refs.append(phi_reference(d["phi_profile"]))
    t0 = time.perf_counter()
    for t in range(0, steps + 1, every):
        if t:
            lat.step(every)
        for m, wl in enumerate(wls):
            d = lat.diagnostics(m, profile=True, check_finite=False)
            s = out[m]
            s["t"].append(t)
            for k in ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2"):
                s[k].append(d[k])
            s["h"].append(lb.mixing_width(d["phi_profile"], phi_refs[m], TRIM))
            if budget:
                b = lat.energy_budget(m)
                for k in BUDGET_KEYS:
                    s[k].append(b[k])
        if t and t % (steps // 4) == 0:
            log(f"{tag}: t = {t} ({time.perf_counter() - t0:.1f} s)")
    final = []
    for m in range(n):
        f = lat.fields(m)
        final.append({k: f[k].cpu().numpy() for k in ("rhoA", "rhoB")})
    _close(lat)
    return out, final


def reduced_precision(lb, inputs, stream, log, steps=20000, every=100):
    res = {}
    for wl in inputs.PRECISION_4096x2048:
        modes = {}
        ref_series, ref_final = _series(lb, [wl], lb.F64, stream, steps, every, log, f"{wl.name} f64")
        r = ref_series[0]
        h64 = np.array(r["h"])
        # 16-bit codes shifted by w_i times the mean density (the default), and
        # unshifted ("-noshift"): floats keep relative precision, so the shift
        # helps the majority phase of a component and hurts its trace phase
        for name, st, r0 in (("f32", lb.F32, 0.0), ("f16s", lb.F16S, 0.0), ("bf16s", lb.BF16S, 0.0),
                             ("f16s-noshift", lb.F16S, -1.0), ("bf16s-noshift", lb.BF16S, -1.0)):
            ser, fin = _series(lb, [wl], st, stream, steps, every, log, f"{wl.name} {name}", (r0, r0))
            s = ser[0]
            mA, mB = np.array(s["mass_A"]), np.array(s["mass_B"])
            h = np.array(s["h"])
            modes[name] = {
                "mass_drift_A": float(np.max(np.abs(mA - mA[0])) / mA[0]),
                "mass_drift_B": float(np.max(np.abs(mB - mB[0])) / mB[0]),
                "mixing_width_final": float(h[-1]),
                "mixing_width_max_abs_err": float(np.max(np.abs(h - h64))),
                "mixing_width_rel_err_final": float(abs(h[-1] - h64[-1]) / max(h64[-1], 1e-30)),
                "rel_l2_rhoA_final": _rel_l2(fin[0]["rhoA"], ref_final[0]["rhoA"]),
                "rel_l2_rhoB_final": _rel_l2(fin[0]["rhoB"], ref_final[0]["rhoB"]),
                "Ek_rel_err_final": float(abs(s["Ek"][-1] - r["Ek"][-1]) / max(abs(r["Ek"][-1]), 1e-30)),
            }
        mA64 = np.array(r["mass_A"])
        res[wl.name] = {"G_AB": wl.G, "steps": steps, "f64_mixing_width_final": float(h64[-1]),
                        "f64_mass_drift_A": float(np.max(np.abs(mA64 - mA64[0])) / mA64[0]),
                        "modes": modes}
    return res


def ensemble_statistics(lb, inputs, stream, log, steps=20000, every=100):
    wls = inputs.ensemble_16()
    t0 = time.perf_counter()
    ser, _ = _series(lb, wls, lb.F32, stream, steps, every, log, "ensemble f32", budget=True)
    wall = time.perf_counter() - t0
    out = {"steps": steps, "every": every, "members": len(wls), "wall_s": round(wall, 1), "groups": {}}
    sample = list(range(0, steps + 1, steps // 10))
    for G in (0.5, 1.5):
        idx = [k for k, wl in enumerate(wls) if wl.G == G]
        grp = {}
        for key in ("h", "Ek", "Ep", "buoyancy") + BUDGET_KEYS:
            a = np.array([ser[k][key] for k in idx])
            grp[key] = {"t": sample,
                        "mean": [float(a[:, t // every].mean()) for t in sample],
                        "std": [float(a[:, t // every].std()) for t in sample]}
        # Eq. 17 over the second half of the run: the change of E_k against
        # the trapezoid integral of -(pb + korteweg + ktau) + viscous -
        # buoyancy (samples every `every` steps), relative to the summed
        # magnitudes of the integrated terms
        res, parts = [], []
        for k in idx:
            s = ser[k]
            t = np.array(s["t"], dtype=np.float64)
            h0 = len(t) // 2
            rhs = np.array([[-s["pb"][j], -s["korteweg"][j], -s["ktau"][j], s["viscous"][j], -s["buoyancy"][j]]
                            for j in range(len(t))])
            integ = np.trapezoid(rhs[h0:], t[h0:], axis=0)
            d_ek = s["Ek"][-1] - s["Ek"][h0]
            res.append(float(abs(d_ek - integ.sum()) / np.sum(np.abs(integ))))
            parts.append(integ)
        grp["balance_residual_rel"] = {"mean": float(np.mean(res)), "max": float(np.max(res))}
        pm = np.mean(np.array(parts), axis=0)
        grp["balance_integrals_second_half"] = dict(zip(("-pb", "-korteweg", "-ktau", "viscous", "-buoyancy"),
                                                        [float(v) for v in pm]))
        grp["members"] = len(idx)
        out["groups"][f"G={G}"] = grp
    return out


def run_all(lb, inputs, stream, log):
    rep = {}
    log("study: FP32 vs FP64 on 10000x5000")
    rep["fp32_vs_fp64_large"] = fp32_vs_fp64_large(lb, inputs, stream, log)
    log("study: 16-bit storage on 4096x2048")
    rep["reduced_precision"] = reduced_precision(lb, inputs, stream, log)
    log("study: 16-member ensemble statistics")
    rep["ensemble_statistics"] = ensemble_statistics(lb, inputs, stream, log)
    return rep
