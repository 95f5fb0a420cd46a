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
  buoyancy), per coupling, and how well Eq. 17 closes per member; the
  interface length and the phase component counts, and a fit of the Korteweg
  flux against the rate of change of interface length (Eq. 21).
* paper_runs: ensembles at the paper's own parameters (Sec. 2: 10^4 x 5 10^3,
  tau = 0.53, g = 9e-6, bulk total density 1.10, G = 0.1381 immiscible or
  0.0805 miscible, the equilibrium immiscible interface with a white-noise
  deformation of amplitude 4, 90000 steps): every 1000 steps the energies,
  all kinetic-energy balance terms, the interface length, the component
  counts and the mixing width of every member.
* surface_tension: at G = 1.5, tau = 1, the Korteweg part of the surface
  tension kappa int (dphi/dy)^2 dy of a relaxed flat interface and the full
  surface tension from Laplace's law on static drops (Eq. 12 pressure), the
  references for the Eq. 21 fit.
"""
from __future__ import annotations

import time

import numpy as np

TRIM = 10


def _lattice(lb, wls, storage, stream):
    members = []
    for wl in wls:
        rA, rB = wl.densities()
        members.append(lb.Member(wl.nx, wl.ny, rA, rB, tau=(wl.tau, wl.tau), G=wl.G, g=wl.gravity))
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


def _series(lb, wls, storage, stream, steps, every, log, tag, budget=False):
    lat = _lattice(lb, wls, storage, stream)
    n = len(wls)
    keys = ["t", "mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2", "h"]
    if budget:
        keys += list(BUDGET_KEYS) + ["length", "comp_A", "comp_B"]
    out = [{k: [] for k in keys} for _ in range(n)]
    t0 = time.perf_counter()
    for t in range(0, steps + 1, every):
        if t:
            lat.step(every)
        for m, wl in enumerate(wls):
            d = lat.diagnostics(m, check_finite=False)
            s = out[m]
            s["t"].append(t)
            for k in ("mass_A", "mass_B", "Ek", "Ep", "buoyancy", "omega2"):
                s[k].append(d[k])
            s["h"].append(lat.mixing_width(m)["width"])
            if budget:
                b = lat.energy_budget(m)
                for k in BUDGET_KEYS:
                    s[k].append(b[k])
                s["length"].append(lat.interface_length(m)["length"])
                c = lat.components(m)
                s["comp_A"].append(c["A"])
                s["comp_B"].append(c["B"])
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
        for name, st in (("f32", lb.F32), ("f16s", lb.F16S), ("bf16s", lb.BF16S)):
            ser, fin = _series(lb, [wl], st, stream, steps, every, log, f"{wl.name} {name}")
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
        for key in ("h", "Ek", "Ep", "buoyancy") + BUDGET_KEYS + ("length", "comp_A", "comp_B"):
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
        # Eq. 21: <u . div P^K> against (1/D) dL/dt (centred differences of
        # the length series); least-squares slope = effective surface tension
        # and the correlation of the two series, per member, after the first
        # tenth of the run
        fits = []
        for k in idx:
            s = ser[k]
            t = np.array(s["t"], dtype=np.float64)
            area = wls[k].nx * (wls[k].ny - 2 * TRIM)
            dl = np.gradient(np.array(s["length"]), t) / area
            kf = np.array(s["korteweg"])
            sel = t >= steps // 10
            x, y = dl[sel], kf[sel]
            slope = float(np.dot(x, y) / max(np.dot(x, x), 1e-300))
            corr = float(np.corrcoef(x, y)[0, 1]) if np.std(x) > 0 and np.std(y) > 0 else float("nan")
            fits.append((slope, corr))
        grp["eq21_gamma_fit"] = {"mean": float(np.mean([f[0] for f in fits])),
                                 "per_member": [round(f[0], 5) for f in fits]}
        grp["eq21_correlation"] = {"mean": float(np.mean([f[1] for f in fits])),
                                   "per_member": [round(f[1], 3) for f in fits]}
        grp["members"] = len(idx)
        out["groups"][f"G={G}"] = grp
    return out


def surface_tension(lb, stream, log, G=1.5, tau=1.0, steps=20000):
    """Korteweg surface tension of a flat interface and Laplace surface
    tension of static drops at (G, tau), from relaxed lattice states."""
    cs2 = 1.0 / 3.0
    kappa = cs2 * cs2 * G / 4.0
    out = {"G": G, "tau": tau, "steps": steps}
    # flat: periodic in y, the A-rich slab in the middle half (two interfaces)
    nx, ny = 16, 256
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    s_ = 0.5 * (np.tanh((y - ny / 4) / 1.5) - np.tanh((y - 3 * ny / 4) / 1.5))
    rA, rB = 0.05 + 1.0 * s_, 0.05 + 1.0 * (1 - s_)
    lat = lb.Lattice([lb.Member(nx, ny, rA, rB, tau=(tau, tau), G=G)], bc_y=lb.PERIODIC_Y, stream=stream,
                     graph_chunk=100, diag_trim=2)
    lat.step(steps)
    f = lat.fields(0)
    phi = (f["rhoA"] - f["rhoB"]).cpu().numpy().mean(axis=1)
    _close(lat)
    dphi = 0.5 * (np.roll(phi, -1) - np.roll(phi, 1))
    out["gamma_korteweg"] = float(kappa * np.sum(dphi * dphi) / 2.0)
    # drops in a periodic box: Laplace's law dp = sigma / R
    n = 256
    radii, dps = [], []
    for R in (24.0, 32.0, 48.0):
        x = np.arange(n)[None, :] - n / 2 + 0.5
        yy = np.arange(n)[:, None] - n / 2 + 0.5
        s_ = 0.5 * (1 - np.tanh((np.hypot(x, yy) - R) / 1.5))
        rA, rB = 0.05 + 1.0 * s_, 0.05 + 1.0 * (1 - s_)
        lat = lb.Lattice([lb.Member(n, n, rA, rB, tau=(tau, tau), G=G)], bc_y=lb.PERIODIC_Y, stream=stream,
                         graph_chunk=100, diag_trim=2)
        lat.step(steps)
        f = {k: v.cpu().numpy() for k, v in lat.fields(0).items()}
        _close(lat)
        p = cs2 * (f["rhoA"] + f["rhoB"]) + G * cs2 * f["rhoA"] * f["rhoB"]   # Eq. 12
        c = n // 2
        p_in = p[c - 3:c + 3, c - 3:c + 3].mean()
        p_out = np.concatenate([p[:6, :].ravel(), p[-6:, :].ravel()]).mean()
        # radius of the relaxed drop from its area
        radii.append(float(np.sqrt(np.count_nonzero(f["rhoA"] > f["rhoB"]) / np.pi)))
        dps.append(float(p_in - p_out))
        log(f"surface tension: drop R = {radii[-1]:.2f}: dp = {dps[-1]:.4e}")
    inv = 1.0 / np.array(radii)
    sigma, icpt = np.polyfit(inv, np.array(dps), 1)
    out["sigma_laplace"] = float(sigma)
    out["laplace_intercept"] = float(icpt)
    out["drops"] = {"R": radii, "dp": dps}
    return out


PAPER = {"nx": 10000, "ny": 5000, "tau": 0.53, "g": 9e-6, "rho_total": 1.10, "steps": 90000,
         "G": {"immiscible": 0.1381, "miscible": 0.0805}}


def equilibrium_profile(lb, stream, log, G=0.1381, tau=0.53, rho_total=1.10, steps=30000):
    """The relaxed flat interface of the immiscible model (Sec. 2): a column
    periodic in y with an A-rich slab in its middle half, relaxed for `steps`
    steps; returns the offsets from the lower interface (B-rich below, A-rich
    above) and the row-mean densities there, and the bulk values."""
    nx, ny = 8, 512
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    s_ = 0.5 * (np.tanh((y - ny / 4) / 1.5) - np.tanh((y - 3 * ny / 4) / 1.5))
    maj, mnr = rho_total / 1.1, rho_total * 0.1 / 1.1
    rA = mnr + (maj - mnr) * s_
    rB = mnr + (maj - mnr) * (1.0 - s_)
    lat = lb.Lattice([lb.Member(nx, ny, rA, rB, tau=(tau, tau), G=G)], bc_y=lb.PERIODIC_Y, stream=stream,
                     graph_chunk=100, diag_trim=2)
    lat.step(steps)
    f = {k: v.cpu().numpy().mean(axis=1) for k, v in lat.fields(0).items()}
    _close(lat)
    phi = f["rhoA"] - f["rhoB"]
    lo = ny // 4 - 60
    j = lo + int(np.argmax(phi[lo:ny // 2] > 0.0))          # first row above the lower interface
    yc = (j - 1) + (-phi[j - 1]) / (phi[j] - phi[j - 1])     # phi = 0 by linear interpolation
    rows = np.arange(ny // 4 - 60, ny // 4 + 60)
    prof = {"y": (rows - yc).tolist(), "rhoA": f["rhoA"][rows].tolist(), "rhoB": f["rhoB"][rows].tolist(),
            "bulk_A_phase": [float(f["rhoA"][ny // 2]), float(f["rhoB"][ny // 2])],
            "bulk_B_phase": [float(f["rhoA"][0]), float(f["rhoB"][0])]}
    log(f"equilibrium profile: A phase (rho_A, rho_B) = {prof['bulk_A_phase']}, "
        f"B phase = {prof['bulk_B_phase']}")
    return prof


def paper_runs(lb, inputs, stream, log, case="immiscible", members=5, seed0=0, storage=None, steps=None,
               every=1000):
    """Ensemble at the paper's parameters (module doc); returns the series."""
    P = PAPER
    steps = P["steps"] if steps is None else steps
    storage = lb.F32 if storage is None else storage
    G = P["G"][case]
    prof = equilibrium_profile(lb, stream, log, tau=P["tau"], rho_total=P["rho_total"])
    yp, pa, pb = (np.array(prof[k]) for k in ("y", "rhoA", "rhoB"))
    mem = []
    for k in range(members):
        h = inputs.white_noise_height(P["nx"], P["ny"], seed0 + k, 4.0)
        rA, rB = inputs.profile_densities(P["nx"], P["ny"], h, yp, pa, pb)
        mem.append(lb.Member(P["nx"], P["ny"], rA, rB, tau=(P["tau"], P["tau"]), G=G,
                             g=((0.0, -P["g"]), (0.0, P["g"]))))
        del rA, rB
    lat = lb.Lattice(mem, forcing=lb.FORCE_SHIFT, storage=storage, graph_chunk=100, stream=stream, diag_trim=TRIM)
    log(f"paper runs {case}: {members} members, steps per pass {lat.steps_per_pass}, tile {lat.tile_shape(0)}")
    keys = ("t", "Ek", "Ep", "buoyancy", "omega2", "pb", "korteweg", "ktau", "viscous", "eta", "length",
            "comp_A", "comp_B", "h", "mass_A", "mass_B", "umax")
    ser = [{k: [] for k in keys} for _ in range(members)]
    t0 = time.perf_counter()
    for t in range(0, steps + 1, every):
        if t:
            lat.step(every)
        for m in range(members):
            d = lat.diagnostics(m, check_finite=False)
            b = lat.energy_budget(m)
            il = lat.interface_length(m)
            c = lat.components(m)
            s = ser[m]
            s["t"].append(t)
            for k in ("Ek", "Ep", "buoyancy", "omega2", "mass_A", "mass_B", "umax"):
                s[k].append(d[k])
            for k in ("pb", "korteweg", "ktau", "viscous", "eta"):
                s[k].append(b[k])
            s["length"].append(il["length"])
            s["comp_A"].append(c["A"])
            s["comp_B"].append(c["B"])
            s["h"].append(lat.mixing_width(m)["width"])
        if t and t % (10 * every) == 0:
            log(f"paper runs {case}: t = {t} ({time.perf_counter() - t0:.0f} s)")
    _close(lat)
    return {"case": case, "G": G, "params": P, "storage": lb.STORAGE_NAMES[storage], "seed0": seed0,
            "every": every, "profile": prof, "wall_s": round(time.perf_counter() - t0, 1), "members": ser}


def run_all(lb, inputs, stream, log):
    rep = {}
    log("study: FP32 vs FP64 on 10000x5000")
    rep["fp32_vs_fp64_large"] = fp32_vs_fp64_large(lb, inputs, stream, log)
    log("study: 16-bit storage on 4096x2048")
    rep["reduced_precision"] = reduced_precision(lb, inputs, stream, log)
    log("study: 16-member ensemble statistics")
    rep["ensemble_statistics"] = ensemble_statistics(lb, inputs, stream, log)
    log("study: surface tension at G = 1.5, tau = 1")
    rep["surface_tension"] = surface_tension(lb, stream, log)
    return rep


SUMMARY_KEYS = ("h", "Ek", "Ep", "length", "comp_A", "comp_B", "umax", "viscous", "korteweg", "buoyancy")


def _finite_until(series) -> int:
    """Index of the last sample up to which every quantity of a member is
    finite (-1 if the first sample is not)."""
    last = -1
    for j in range(len(series["t"])):
        if all(np.isfinite(series[k][j]) for k in SUMMARY_KEYS if k in series):
            last = j
        else:
            break
    return last


def paper_analysis(members, nx, ny, t_from=10000, t_fit=20000, t_peak_until=50000) -> dict:
    """Derived statistics of paper-parameter series (members: the series of
    the members finite to the end of the run; the topology entry also takes
    failed members up to their last finite sample if they are passed):

    * Eq. 17: over [t_from, end] the change of E_k against the trapezoid
      integral of -(p_b + Korteweg + K^(tau) fluxes) + viscous - buoyancy;
      residual relative to the summed magnitudes of the integrated terms
      (mean and largest over the members) and the member-mean integrals.
    * Eq. 22: largest relative difference between the viscous term and
      -eta <omega^2> from t_fit on: the median and largest per-sample
      relative difference and the range over the members of the ratio of
      their time integrals.
    * Topology: per member the first sample at which either phase has more
      than one connected component.
    * Interface growth: the rate dL/dt of the member-mean interface length
      (centred differences), its peak up to t_peak_until and the first local
      minimum after that peak.
    * Eq. 21: per member the least-squares slope of <u . div P^K> against
      (dL/dt) / D (D the averaging area, rows [TRIM, ny - TRIM)) from t_fit
      on, and the correlation of the two series."""
    out = {"members": len(members)}
    need = ("t", "Ek", "pb", "korteweg", "ktau", "viscous", "buoyancy", "eta", "omega2", "length")
    if not members or any(k not in members[0] for k in need):
        return out
    t = np.array(members[0]["t"], dtype=np.float64)
    j0 = int(np.searchsorted(t, t_from))
    res, parts = [], []
    for s in members:
        rhs = np.stack([-np.array(s["pb"]), -np.array(s["korteweg"]), -np.array(s["ktau"]),
                        np.array(s["viscous"]), -np.array(s["buoyancy"])], axis=1)
        integ = np.trapezoid(rhs[j0:], t[j0:], axis=0)
        d_ek = s["Ek"][-1] - s["Ek"][j0]
        res.append(float(abs(d_ek - integ.sum()) / np.sum(np.abs(integ))))
        parts.append(integ)
    out["eq17_residual_rel"] = {"mean": float(np.mean(res)), "max": float(np.max(res)), "from_t": int(t[j0])}
    out["eq17_integrals"] = dict(zip(("-pb", "-korteweg", "-ktau", "viscous", "-buoyancy"),
                                     [float(v) for v in np.mean(np.array(parts), axis=0)]))
    jf = int(np.searchsorted(t, t_fit))
    rel, ratio = [], []
    for s in members:
        v = np.array(s["viscous"][jf:])
        e = np.array(s["eta"][jf:]) * np.array(s["omega2"][jf:])
        rel.append(np.abs(v + e) / np.abs(e))
        ratio.append(float(np.trapezoid(v, t[jf:]) / np.trapezoid(-e, t[jf:])))
    out["eq22"] = {"median_rel_diff": float(np.median(np.concatenate(rel))),
                   "max_rel_diff": float(np.max(np.concatenate(rel))),
                   "integral_ratio_min": float(np.min(ratio)), "integral_ratio_max": float(np.max(ratio)),
                   "from_t": int(t[jf])}
    mean_len = np.mean(np.array([s["length"] for s in members]), axis=0)
    rate = np.gradient(mean_len, t)
    sel = np.nonzero(t <= t_peak_until)[0]
    jp = int(sel[np.argmax(rate[sel])])
    jm = jp
    while jm + 1 <= sel[-1] and rate[jm + 1] <= rate[jm]:   # first local minimum after the peak
        jm += 1
    out["length_rate"] = {"peak_t": int(t[jp]), "peak": float(rate[jp]), "dip_t": int(t[jm]), "dip": float(rate[jm])}
    area = nx * (ny - 2 * TRIM)
    slopes, corrs = [], []
    for s in members:
        x = np.gradient(np.array(s["length"]), t)[jf:] / area
        y = np.array(s["korteweg"][jf:])
        slopes.append(float(np.dot(x, y) / max(np.dot(x, x), 1e-300)))
        corrs.append(float(np.corrcoef(x, y)[0, 1]) if np.std(x) > 0 and np.std(y) > 0 else float("nan"))
    out["eq21_gamma_fit"] = {"mean": float(np.mean(slopes)), "std": float(np.std(slopes)),
                             "correlation_mean": float(np.mean(corrs)), "from_t": int(t[jf])}
    return out


def _first_split(s) -> int | None:
    """Time of the first sample with more than one component in either phase."""
    for j, tj in enumerate(s["t"]):
        if not (np.isfinite(s["comp_A"][j]) and np.isfinite(s["comp_B"][j])):
            return None
        if s["comp_A"][j] > 1 or s["comp_B"][j] > 1:
            return int(tj)
    return None


def summarise_paper_runs(runs, times=None) -> dict:
    """Ensemble tables of paper-parameter runs (the output of paper_runs, one
    or more files per case): per case and sample time, the mean and standard
    deviation over (a) the members that stay finite to the end of the run
    and (b) every member still finite at that time (members that fail are
    included up to their last finite sample), so the effect of dropping the
    failed members on each statistic is visible; per member the time of its
    last finite sample and of its first topology change; and the derived
    statistics of paper_analysis over the members finite to the end."""
    by_case = {}
    for r in runs:
        c = by_case.setdefault(r["case"], {"G": r["G"], "storage": r["storage"], "members": [], "seeds": [],
                                           "nx": r.get("params", PAPER)["nx"], "ny": r.get("params", PAPER)["ny"]})
        for k, ser in enumerate(r["members"]):
            c["members"].append(ser)
            c["seeds"].append(r["seed0"] + k)
    out = {}
    for case, c in by_case.items():
        mem = c["members"]
        t_all = mem[0]["t"]
        sel = times or [t for t in t_all if t and t % 10000 == 0]
        last = [_finite_until(ser) for ser in mem]
        end = len(t_all) - 1
        rows = {}
        for t in sel:
            j = t_all.index(t)
            row = {}
            for k in SUMMARY_KEYS:
                if k not in mem[0]:
                    continue
                surv = [ser[k][j] for ser, l in zip(mem, last) if l == end]
                alive = [ser[k][j] for ser, l in zip(mem, last) if l >= j]
                row[k] = {"survivors": {"mean": float(np.mean(surv)) if surv else None,
                                        "std": float(np.std(surv)) if surv else None, "n": len(surv)},
                          "finite_at_t": {"mean": float(np.mean(alive)) if alive else None,
                                          "std": float(np.std(alive)) if alive else None, "n": len(alive)}}
            rows[str(t)] = row
        out[case] = {"G": c["G"], "storage": c["storage"], "members": len(mem),
                     "finite_to_end": sum(1 for l in last if l == end),
                     "last_finite_t": {str(s): (t_all[l] if l >= 0 else None) for s, l in zip(c["seeds"], last)},
                     "first_split_t": {str(s): _first_split(ser) for s, ser in zip(c["seeds"], mem)},
                     "tables": rows,
                     "analysis": paper_analysis([ser for ser, l in zip(mem, last) if l == end], c["nx"], c["ny"])}
    return out


# (key, row label, divisor, decimals) of the markdown tables
TABLE_ROWS = (("h", "mixing width h", 1.0, 0), ("Ek", "E_k (10⁻⁴)", 1e-4, 2), ("Ep", "E_p (10⁻³)", 1e-3, 2),
              ("length", "interface length L (10³)", 1e3, 1), ("comp_A", "components of A", 1.0, 0),
              ("comp_B", "components of B", 1.0, 0), ("umax", "max\\|u\\|", 1.0, 3))


def paper_tables_markdown(summary) -> str:
    """Markdown tables of a paper_runs summary: per case, one row per quantity
    and member set (those finite to the end; every member finite at t), each
    cell the mean ± standard deviation and, where it is not every member, the
    member count in brackets."""
    out = []
    for case, c in summary.items():
        times = list(c["tables"])
        out.append(f"{case} (G = {c['G']}, {c['storage']}; {c['finite_to_end']} of {c['members']} members "
                   f"finite to the end):\n")
        out.append("| quantity | members | " + " | ".join(f"{int(t):,}".replace(",", " ") for t in times) + " |")
        out.append("|---|---|" + "---|" * len(times))
        for key, label, div, dec in TABLE_ROWS:
            if key not in c["tables"][times[0]]:
                continue
            for sel, name in (("survivors", "finite to end"), ("finite_at_t", "finite at t")):
                cells = []
                for t in times:
                    s = c["tables"][t][key][sel]
                    if s["mean"] is None:
                        cells.append("–")
                        continue
                    cell = f"{s['mean'] / div:.{dec}f} ± {s['std'] / div:.{dec}f}"
                    if s["n"] != c["members"]:
                        cell += f" [{s['n']}]"
                    cells.append(cell)
                out.append(f"| {label} | {name} | " + " | ".join(cells) + " |")
        failed = {s: t for s, t in c["last_finite_t"].items() if t != int(times[-1])}
        out.append("")
        out.append("last finite sample of the failed members (seed: t): " +
                   (", ".join(f"{s}: {t}" for s, t in failed.items()) if failed else "none"))
        splits = [t for t in c.get("first_split_t", {}).values() if t is not None]
        if splits:
            out.append(f"first topology change: t = {min(splits)} … {max(splits)} ({len(splits)} members)")
        a = c.get("analysis", {})
        if "eq17_residual_rel" in a:
            r, i = a["eq17_residual_rel"], a["eq17_integrals"]
            out.append(f"Eq. 17 from t = {r['from_t']} (members finite to the end): residual {r['mean']:.2e} of the "
                       f"summed integrated terms (largest {r['max']:.2e}); integrals " +
                       ", ".join(f"{k} {v:.3e}" for k, v in i.items()))
            e = a["eq22"]
            out.append(f"Eq. 22 from t = {e['from_t']}: viscous vs -eta<omega^2> per sample median "
                       f"{e['median_rel_diff']:.2%} (largest {e['max_rel_diff']:.1%}); ratio of the time integrals "
                       f"{e['integral_ratio_min']:.4f} … {e['integral_ratio_max']:.4f}")
            lr = a["length_rate"]
            out.append(f"dL/dt of the mean length: peak {lr['peak']:.2f} at t = {lr['peak_t']}, then down to "
                       f"{lr['dip']:.2f} at t = {lr['dip_t']}")
            g = a["eq21_gamma_fit"]
            out.append(f"Eq. 21 fit: gamma_eff = {g['mean']:.5f} ± {g['std']:.5f} (correlation "
                       f"{g['correlation_mean']:.2f})")
        out.append("")
    return "\n".join(out)


def main(argv):
    """python -m paper_2101_04847_amd.studies paper-runs CASE MEMBERS SEED0 OUT.json [STEPS [STORAGE]]
    python -m paper_2101_04847_amd.studies paper-summary OUT.json RUN.json [RUN.json ...]
    python -m paper_2101_04847_amd.studies paper-tables SUMMARY.json"""
    import json
    import sys as _sys

    if len(argv) >= 3 and argv[0] == "paper-summary":
        runs = []
        for path in argv[2:]:
            with open(path) as fh:
                runs.append(json.load(fh))
        with open(argv[1], "w") as fh:
            json.dump(summarise_paper_runs(runs), fh, indent=1)
        print(json.dumps({"out": argv[1], "runs": len(runs)}))
        return
    if len(argv) == 2 and argv[0] == "paper-tables":
        with open(argv[1]) as fh:
            print(paper_tables_markdown(json.load(fh)))
        return

    import torch

    from paper_2101_04847_amd import inputs, lb

    if len(argv) < 5 or argv[0] != "paper-runs":
        raise SystemExit(main.__doc__)

    def log(*a):
        print("[study]", *a, file=_sys.stderr, flush=True)

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    steps = int(argv[5]) if len(argv) > 5 and int(argv[5]) > 0 else None
    storage = {"f64": lb.F64, "f32": lb.F32}[argv[6]] if len(argv) > 6 else None
    rep = paper_runs(lb, inputs, stream, log, case=argv[1], members=int(argv[2]), seed0=int(argv[3]), steps=steps,
                     storage=storage)
    with open(argv[4], "w") as fh:
        json.dump(rep, fh)
    print(json.dumps({"out": argv[4], "case": rep["case"], "members": len(rep["members"]), "wall_s": rep["wall_s"]}))


if __name__ == "__main__":
    import sys
    main(sys.argv[1:])
